// Linkage model for parallel variation (Sec. 4.2.1): the edges of the mesh
// are the FOS elements; a greedy set cover keeps a subset of edges that
// covers every point; two elements interact when their dependent tetrahedra
// (the tets holding one of their points) overlap; DSATUR colours the
// interaction graph, so the elements of one colour can be varied and
// evaluated in parallel (one batched partial evaluation per colour).
//
// Definitions where the paper names the algorithms only:
//   set cover: greedy, the edge covering the most uncovered points first,
//     ties to the lexicographically smallest (a, b), a < b; with edges this
//     is one ascending pass taking edges with two uncovered ends, then one
//     taking edges with one; points in no tet stay uncovered;
//   DSATUR: repeatedly the uncoloured element with the most distinct colours
//     among its neighbours, ties to the larger degree, then the smaller
//     index, gets the smallest colour none of its neighbours has.
// Host code only.
#include <algorithm>
#include <utility>
#include <vector>

#include "morea_internal.h"

extern "C" morea_status morea_build_fos(int32_t n_points, int32_t n_tets, const int32_t* tets, int32_t capacity,
                                        int32_t* elem_pts, int32_t* color, int32_t* n_elements, int32_t* n_colors) {
  if (n_points < 1 || n_tets < 0 || (n_tets > 0 && !tets) || !elem_pts || !color || !n_elements || !n_colors) {
    morea::set_error("bad argument");
    return MOREA_EINVAL;
  }
  for (int64_t i = 0; i < 4 * static_cast<int64_t>(n_tets); i++)
    if (tets[i] < 0 || tets[i] >= n_points) {
      morea::set_error("tet vertex index out of range");
      return MOREA_EINVAL;
    }
  // mesh edges, ascending
  std::vector<std::pair<int, int>> edges;
  edges.reserve(6 * static_cast<size_t>(n_tets));
  for (int t = 0; t < n_tets; t++)
    for (int i = 0; i < 4; i++)
      for (int j = i + 1; j < 4; j++) {
        const int a = tets[4 * t + i], b = tets[4 * t + j];
        if (a != b) edges.emplace_back(std::min(a, b), std::max(a, b));
      }
  std::sort(edges.begin(), edges.end());
  edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
  // greedy set cover
  std::vector<char> covered(n_points, 0);
  std::vector<std::pair<int, int>> chosen;
  for (int pass = 2; pass >= 1; pass--)
    for (const auto& e : edges) {
      const int fresh = !covered[e.first] + !covered[e.second];
      if (fresh >= pass) {
        chosen.push_back(e);
        covered[e.first] = covered[e.second] = 1;
      }
    }
  const int n = static_cast<int>(chosen.size());
  if (n > capacity) {
    morea::set_error("more FOS elements than the capacity");
    return MOREA_ERANGE;
  }
  // interaction graph: elements with a point in a common tet
  std::vector<std::vector<int>> of_point(n_points);
  for (int k = 0; k < n; k++) {
    of_point[chosen[k].first].push_back(k);
    of_point[chosen[k].second].push_back(k);
  }
  std::vector<std::vector<int>> adj(n);
  for (int t = 0; t < n_tets; t++) {
    std::vector<int> here;
    for (int i = 0; i < 4; i++)
      for (int k : of_point[tets[4 * t + i]]) here.push_back(k);
    std::sort(here.begin(), here.end());
    here.erase(std::unique(here.begin(), here.end()), here.end());
    for (size_t x = 0; x < here.size(); x++)
      for (size_t y = 0; y < here.size(); y++)
        if (x != y) adj[here[x]].push_back(here[y]);
  }
  for (auto& a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  // DSATUR
  std::vector<int> col(n, -1);
  std::vector<std::vector<char>> seen(n);   // colours present among the neighbours
  std::vector<int> sat(n, 0);
  int used = 0;
  for (int step = 0; step < n; step++) {
    int v = -1;
    for (int k = 0; k < n; k++) {
      if (col[k] >= 0) continue;
      if (v < 0 || sat[k] > sat[v] || (sat[k] == sat[v] && adj[k].size() > adj[v].size())) v = k;
    }
    int c = 0;
    while (c < static_cast<int>(seen[v].size()) && seen[v][c]) c++;
    col[v] = c;
    used = std::max(used, c + 1);
    for (int u : adj[v]) {
      if (static_cast<int>(seen[u].size()) <= c) seen[u].resize(c + 1, 0);
      if (!seen[u][c]) {
        seen[u][c] = 1;
        sat[u] += 1;
      }
    }
  }
  for (int k = 0; k < n; k++) {
    elem_pts[2 * k] = chosen[k].first;
    elem_pts[2 * k + 1] = chosen[k].second;
    color[k] = col[k];
  }
  *n_elements = n;
  *n_colors = used;
  return MOREA_OK;
}
