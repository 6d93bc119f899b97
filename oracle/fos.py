"""Linkage model of the optimizer's parallel variation -- plain reference,
test infrastructure only.  Sec. 4.2.1: edges of the mesh as FOS elements, a
greedy set cover selecting edges that cover every point, an interaction graph
joining elements whose dependent tetrahedra overlap, DSATUR (Brelaz) colouring
into groups that are varied and evaluated in parallel.

Readings where the paper names the algorithms only (listed in the design
notes): the greedy set cover takes the edge covering the most uncovered
points, ties to the lexicographically smallest (a, b); DSATUR takes the
uncoloured vertex of largest saturation (distinct colours among its
neighbours), ties to the larger degree, then the smaller index, and gives it
the smallest colour absent from its neighbours.
"""


def mesh_edges(tets):
    return sorted({(min(int(a), int(b)), max(int(a), int(b)))
                   for tv in tets for i, a in enumerate(tv) for b in list(tv)[i + 1:] if a != b})


def greedy_set_cover(n_points, edges):
    """Greedy cover of the points by edges: repeatedly the edge with the most
    uncovered end points (lexicographically smallest among equals)."""
    uncovered = set()
    for a, b in edges:
        uncovered.update((a, b))
    chosen = []
    remaining = list(edges)
    while True:
        best, gain = None, 0
        for e in remaining:
            g = (e[0] in uncovered) + (e[1] in uncovered)
            if g > gain:
                best, gain = e, g
                if g == 2:
                    break
        if best is None:
            return chosen
        chosen.append(best)
        uncovered.discard(best[0])
        uncovered.discard(best[1])
        remaining = [e for e in remaining if e != best and ((e[0] in uncovered) or (e[1] in uncovered))]


def interaction_graph(tets, elements):
    """Elements i, j are joined when their dependent tets (the tets holding
    one of their points) overlap."""
    holding = {}
    for t, tv in enumerate(tets):
        for v in tv:
            holding.setdefault(int(v), set()).add(t)
    deps = [holding.get(a, set()) | holding.get(b, set()) for a, b in elements]
    users = {}
    for i, d in enumerate(deps):
        for t in d:
            users.setdefault(t, []).append(i)
    adj = [set() for _ in elements]
    for members in users.values():
        for i in members:
            adj[i].update(members)
    return [sorted(a - {i}) for i, a in enumerate(adj)]


def dsatur(adj):
    """Colour of every vertex (Brelaz's DSATUR)."""
    n = len(adj)
    color = [-1] * n
    for _ in range(n):
        def key(v):
            sat = len({color[u] for u in adj[v] if color[u] >= 0})
            return (sat, len(adj[v]), -v)
        v = max((v for v in range(n) if color[v] < 0), key=key)
        taken = {color[u] for u in adj[v]}
        c = 0
        while c in taken:
            c += 1
        color[v] = c
    return color


def build(n_points, tets):
    """(elements [(a, b)], colours) of a mesh."""
    elements = greedy_set_cover(n_points, mesh_edges(tets))
    return elements, dsatur(interaction_graph(tets, elements))
