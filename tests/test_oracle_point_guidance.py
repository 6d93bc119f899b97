"""Pins of the oracle's point-based guidance error (the prior work's form
that Sec. 4.1.3 replaces): zero when the meshes carry C_s exactly onto C_t,
|t|^2 for a translation of well-separated points, a floating-point brute
force (locate each point by solving barycentric coordinates in every tet,
map, take the nearest target point) on perturbed candidates, and points
outside the mesh left out and counted."""
import numpy as np

import oracle
import synth


def problem_with_sets(p, src, tgt):
    return oracle.Problem(p.dims, p.image_src, p.image_tgt, p.tets, p.ref_points, p.elasticity, src, tgt,
                          p.radius)


def cand(S, T):
    return np.ascontiguousarray(np.stack([np.asarray(S, np.float32).T, np.asarray(T, np.float32).T]))[None]


def grid(points):
    return (np.rint(np.asarray(points, np.float64) * 1024) / 1024).astype(np.float32)


def test_exact_affine_warp_gives_zero():
    p = synth.make_problem(1)
    rs = np.random.default_rng(0)
    # on a 1/32 grid, so that their images under A (entries multiples of 1/32)
    # lie exactly on the 2^-10 grid
    src = [(np.rint(rs.uniform(2, 29, (n, 3)) * 32) / 32).astype(np.float32) for n in (40, 25)]
    A = np.array([[1.0625, 0.125, 0.0], [-0.0625, 0.9375, 0.0625], [0.0, 0.03125, 1.0]])
    b = np.array([-0.75, 1.25, 0.5])
    c = np.array([15.5, 15.5, 15.5])
    warp = lambda x: ((np.asarray(x, np.float64) - c) @ A.T + c + b).astype(np.float32)
    tgt = [warp(s) for s in src]
    assert all(np.array_equal(grid(t), t) for t in tgt)
    op = problem_with_sets(p, src, tgt)
    f, un = op.point_guidance(cand(p.ref_points, warp(p.ref_points)))
    assert un[0] == 0 and f[0] < 1e-12


def test_translation_of_separated_points():
    p = synth.make_problem(1)
    pts = grid(np.array([[4.25, 5.5, 6.0], [20.0, 8.25, 12.5], [10.5, 24.0, 20.25], [26.0, 26.5, 4.75]]))
    op = problem_with_sets(p, [pts], [pts])
    t = np.array([0.375, -0.25, 0.5], np.float32)
    f, un = op.point_guidance(cand(p.ref_points, p.ref_points + t))
    assert un[0] == 0
    np.testing.assert_allclose(f[0], float(t.astype(np.float64) @ t.astype(np.float64)), rtol=1e-12)


def brute_force(p, src, tgt, c):
    S = np.rint(c[0].T.astype(np.float64) * 1024) / 1024
    T = np.rint(c[1].T.astype(np.float64) * 1024) / 1024
    total, n, unmapped = 0.0, 0, 0
    for cs, ct in zip(src, tgt):
        ct = np.rint(ct.astype(np.float64) * 1024) / 1024
        for x in np.rint(cs.astype(np.float64) * 1024) / 1024:
            hit = None
            for tv in p.tets:
                E = (S[tv[1:]] - S[tv[0]]).T
                lam = np.linalg.solve(E, x - S[tv[0]])
                if lam.min() >= -1e-12 and lam.sum() <= 1 + 1e-12:
                    hit = T[tv[0]] + (T[tv[1:]] - T[tv[0]]).T @ lam
                    break
            if hit is None:
                unmapped += 1
                continue
            total += np.min(np.sum((ct - hit) ** 2, axis=1))
            n += 1
    return total / n, unmapped


def test_perturbed_candidates_against_brute_force():
    p = synth.make_problem(1)
    op = oracle.Problem.from_synth(p)
    pop = synth.make_population(p, pop=3, seed=41, perturb_source=True, fold_fraction=0.0)
    f, un = op.point_guidance(pop)
    for c in range(3):
        want, wun = brute_force(p, p.sets_src, p.sets_tgt, pop[c])
        assert un[c] == wun
        np.testing.assert_allclose(f[c], want, rtol=1e-9)


def test_points_outside_the_mesh_are_counted():
    p = synth.make_problem(1)
    pts = grid(np.array([[4.25, 5.5, 6.0], [-3.0, 5.0, 5.0], [20.0, 8.25, 12.5], [40.0, 2.0, 2.0]]))
    op = problem_with_sets(p, [pts], [pts])
    f, un = op.point_guidance(cand(p.ref_points, p.ref_points))
    assert un[0] == 2 and f[0] == 0.0
    bad = cand(p.ref_points, p.ref_points)
    bad[0, 1, 0, 3] = np.nan
    f, un = op.point_guidance(bad)
    assert np.isnan(f[0]) and un[0] == 0
