"""Pins of the linkage-model reference (Sec. 4.2.1) and parity of the
library's native implementation with it (host code: no GPU needed).

The reference is pinned by what the algorithms guarantee: the cover covers
every point of the mesh with mesh edges and is a maximal matching followed by
single-point edges; DSATUR colours a valid colouring, is optimal on bipartite
graphs, cycles and complete graphs, and gives the Petersen graph 3 colours; the
interaction graph joins exactly the elements whose dependent tets overlap
(brute force over tets)."""
import ctypes
import functools

import numpy as np
import pytest

import synth
from oracle import fos

try:
    import paper_2303_04873_amd as morea
    LIB = morea.load_library()
except (ImportError, OSError):
    LIB = None


@functools.lru_cache(maxsize=None)
def reference(config):
    p = synth.make_problem(config)
    return p, fos.build(p.n_points, p.tets)


def test_dsatur_known_graphs():
    cycle5 = [[(i - 1) % 5, (i + 1) % 5] for i in range(5)]
    assert max(fos.dsatur(cycle5)) + 1 == 3
    cycle6 = [[(i - 1) % 6, (i + 1) % 6] for i in range(6)]
    assert max(fos.dsatur(cycle6)) + 1 == 2
    k4 = [[j for j in range(4) if j != i] for i in range(4)]
    assert sorted(fos.dsatur(k4)) == [0, 1, 2, 3]
    # 4 x 5 grid graph (bipartite)
    grid = [[] for _ in range(20)]
    for r in range(4):
        for c in range(5):
            v = 5 * r + c
            for dr, dc in ((0, 1), (1, 0)):
                if r + dr < 4 and c + dc < 5:
                    u = 5 * (r + dr) + c + dc
                    grid[v].append(u)
                    grid[u].append(v)
    assert max(fos.dsatur(grid)) + 1 == 2
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    petersen = [[] for _ in range(10)]
    for a, b in outer + spokes + inner:
        petersen[a].append(b)
        petersen[b].append(a)
    col = fos.dsatur(petersen)
    assert max(col) + 1 == 3 and all(col[a] != col[b] for a, b in outer + spokes + inner)
    # a hand-traced case: path 0-1-2 plus a triangle 2-3-4
    g = [[1], [0, 2], [1, 3, 4], [2, 4], [2, 3]]
    assert fos.dsatur(g) == [0, 1, 0, 1, 2]


@pytest.mark.parametrize("config", [1, 2])
def test_cover_and_colouring_properties(config):
    p, (elements, colors) = reference(config)
    edges = set(fos.mesh_edges(p.tets))
    assert all(e in edges for e in elements)
    covered = {v for e in elements for v in e}
    assert covered == set(range(p.n_points))
    # the first part is a maximal matching, the rest adds one new point each
    seen, matching = set(), True
    for a, b in elements:
        if matching and (a in seen or b in seen):
            matching = False
        if not matching:
            assert (a in seen) != (b in seen)
        seen.update((a, b))
    # interaction = overlapping dependent tets (brute force), colouring valid
    adj = fos.interaction_graph(p.tets, elements)
    deps = [{t for t, tv in enumerate(p.tets) if a in tv or b in tv} for a, b in elements]
    rs = np.random.default_rng(0)
    for i in rs.choice(len(elements), min(60, len(elements)), replace=False):
        assert set(adj[i]) == {j for j in range(len(elements)) if j != i and deps[i] & deps[j]}
    assert all(colors[i] != colors[j] for i in range(len(elements)) for j in adj[i])


@pytest.mark.skipif(LIB is None, reason="libmorea.so is not built")
@pytest.mark.parametrize("config", [1, 2])
def test_library_matches_reference(config):
    p = synth.make_problem(config)
    tets = np.ascontiguousarray(p.tets, dtype=np.int32)
    cap = p.n_points
    ep = np.empty((cap, 2), np.int32)
    col = np.empty(cap, np.int32)
    ne, nc = ctypes.c_int32(), ctypes.c_int32()
    assert LIB.morea_build_fos(p.n_points, len(tets), tets.ctypes.data_as(ctypes.c_void_p), cap,
                               ep.ctypes.data_as(ctypes.c_void_p), col.ctypes.data_as(ctypes.c_void_p),
                               ctypes.byref(ne), ctypes.byref(nc)) == morea.MOREA_OK
    _, (elements, colors) = reference(config)
    assert ne.value == len(elements) and nc.value == max(colors) + 1
    np.testing.assert_array_equal(ep[:ne.value], np.array(elements, np.int32))
    np.testing.assert_array_equal(col[:ne.value], np.array(colors, np.int32))
    # too small a capacity is refused
    assert LIB.morea_build_fos(p.n_points, len(tets), tets.ctypes.data_as(ctypes.c_void_p), 1,
                               ep.ctypes.data_as(ctypes.c_void_p), col.ctypes.data_as(ctypes.c_void_p),
                               ctypes.byref(ne), ctypes.byref(nc)) == morea.MOREA_ERANGE
