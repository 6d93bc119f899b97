"""Pins of the fold-repair reference (Sec. 4.3.1) against what the geometry
fixes: the step size against a floating-point distance to the neighbours'
centroid, the chosen move against a brute force over the trials of a single
tet, abort and pinned-axis cases, and every applied move's constraint change
against the independent C oracle's severity of the whole candidate."""
import numpy as np

import oracle
import synth
from oracle import repair as R

# one tet: 0, 1, 2 pinned on every axis, point 3 free
TET = np.array([[0, 1, 2, 3]], np.int32)
REF = np.array([[10.0, 10.0, 10.0], [20.0, 10.5, 10.25], [11.0, 21.0, 10.5], [12.0, 12.5, 22.0]], np.float32)
PIN = np.array([7, 7, 7, 0], np.uint8)


def cand_of(points):
    pts = np.asarray(points, np.float32)
    return np.stack([pts.T, pts.T])[None]      # both meshes the same


def pushed():
    """Point 3 mirrored through the plane of 0, 1, 2 (on the grid)."""
    P = REF.copy()
    a, b, c = REF[0].astype(np.float64), REF[1].astype(np.float64), REF[2].astype(np.float64)
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n)
    d = np.dot(REF[3] - a, n)
    P[3] = np.rint((REF[3] - 1.6 * d * n) * 1024) / 1024
    return P


def test_sigma_is_ring_distance_rounded_down_to_a_power_of_two():
    """sigma = 2^floor(log2(|v - centroid of v's neighbours|)) in grid units,
    against a floating-point distance, on random 2x2x2-cell Kuhn meshes."""
    pts, tets, fixed = synth.kuhn_grid((16, 16, 16), (3, 3, 3))
    inc = R.incidence(tets, len(pts))
    rs = np.random.default_rng(0)
    checked = 0
    for _ in range(20):
        P = np.rint((pts + rs.normal(0, 2.0, pts.shape)) * 1024) / 1024
        X = [[int(np.rint(x * 1024)) for x in p] for p in P]
        for v in range(len(P)):
            nb = sorted({int(u) for t in tets if v in t for u in t if u != v})
            dist = np.linalg.norm(P[v] * 1024 - np.mean(P[nb] * 1024, axis=0))
            lg = np.log2(max(dist, 1e-300))
            if abs(lg - round(lg)) < 1e-9:
                continue
            want = 1 if dist < 1 else 2 ** min(int(np.floor(lg)), R.SIGMA_MAX_LOG2)
            assert R.sigma(X, tets, inc[v], v) == want
            checked += 1
    assert checked > 400


def test_single_tet_fold_repaired_by_the_best_trial():
    P = pushed()
    c = cand_of(P)
    rs = np.random.default_rng(1)
    noise = rs.normal(size=(1, 8, 64, 3)).astype(np.float32)
    out, moves, outcome, logs = R.repair(TET, REF, c, noise, fixed=PIN)
    # points 0, 1, 2 cannot move (ties, no abort); point 3 of mesh S uses draw 3
    assert outcome[0] in (R.DONE, R.OUT_OF_DRAWS) and moves[0] >= 1
    log = logs[0]
    assert [(m, v) for m, v, *_ in log[:4]] == [(0, 0), (0, 1), (0, 2), (0, 3)]
    m, v, sg, c0, cb, k = log[3]
    dist = np.linalg.norm(P[3].astype(np.float64) * 1024 - P[:3].astype(np.float64).mean(axis=0) * 1024)
    assert sg == 2 ** int(np.floor(np.log2(dist)))
    # brute force over the 64 trials with floating-point volumes
    base = np.rint(P[3].astype(np.float64) * 1024)
    trials = base + np.rint(sg * noise[0, 3].astype(np.float64))
    ref_sign = np.sign(np.linalg.det((REF[1:] - REF[0]).astype(np.float64)))
    a = P[:3].astype(np.float64) * 1024
    vols = np.array([np.linalg.det(np.stack([a[1] - a[0], a[2] - a[0], t - a[0]])) for t in trials])
    folded = (np.sign(vols) != ref_sign) | (vols == 0)
    key = [(int(f), abs(v) if f else 0.0, i) for i, (f, v) in enumerate(zip(folded, vols))]
    kb = min(key)[2]
    assert k == kb
    np.testing.assert_array_equal(out[0, 0, :, 3], (trials[kb] / 1024).astype(np.float32))
    np.testing.assert_array_equal(out[0, 0, :, :3], c[0, 0, :, :3])


def test_all_trials_worse_aborts_and_leaves_the_candidate():
    P = pushed()
    c = cand_of(P)
    a, b, cc = REF[0].astype(np.float64), REF[1].astype(np.float64), REF[2].astype(np.float64)
    n = np.cross(b - a, cc - a)
    n /= np.linalg.norm(n)
    away = -n if np.dot(REF[3] - a, n) > 0 else n      # further through the face
    noise = np.zeros((1, 4, 64, 3), np.float32)
    noise[0, 3] = (away * np.linspace(0.5, 3.0, 64)[:, None]).astype(np.float32)
    out, moves, outcome, _ = R.repair(TET, REF, c, noise, fixed=PIN)
    assert outcome[0] == R.ABORTED and moves[0] == 0
    np.testing.assert_array_equal(out, c)


def test_pinned_axes_do_not_move_and_draws_run_out():
    P = pushed()
    c = cand_of(P)
    rs = np.random.default_rng(2)
    noise = rs.normal(size=(1, 8, 64, 3)).astype(np.float32)
    pin = PIN.copy()
    pin[3] = 1                                           # x of point 3 pinned
    out, moves, outcome, _ = R.repair(TET, REF, c, noise, fixed=pin)
    assert out[0, 0, 0, 3] == c[0, 0, 0, 3]
    # 3 draws only: points 0, 1, 2 use them up before point 3
    out3, moves3, outcome3, _ = R.repair(TET, REF, c, noise[:, :3], fixed=PIN)
    assert outcome3[0] == R.OUT_OF_DRAWS and moves3[0] == 0


def test_no_fold_and_invalid_candidates_untouched():
    c = cand_of(REF)
    noise = np.zeros((1, 2, 64, 3), np.float32)
    out, moves, outcome, _ = R.repair(TET, REF, c, noise)
    assert outcome[0] == R.NO_FOLD and moves[0] == 0
    bad = cand_of(pushed())
    bad[0, 1, 2, 1] = 600.0
    out, moves, outcome, _ = R.repair(TET, REF, bad, noise)
    assert outcome[0] == R.INVALID
    np.testing.assert_array_equal(out, bad)


def fixed_mask(p):
    return (p.fixed_axes.astype(np.uint8) * np.array([1, 2, 4], np.uint8)).sum(axis=1).astype(np.uint8)


def test_moves_change_the_whole_candidate_by_their_local_constraint():
    """Only the moved point's incident tets change, so the C oracle's severity
    of the whole candidate drops by exactly the local |6V| improvement of the
    applied moves; nothing the repair does increases it."""
    p = synth.make_problem(1)
    pop = synth.make_population(p, pop=16, seed=21, perturb_source=True, fold_fraction=0.5)
    rs = np.random.default_rng(3)
    noise = rs.normal(size=(16, 12, 64, 3)).astype(np.float32)
    out, moves, outcome, logs = R.repair(p.tets, p.ref_points, pop, noise, fixed=fixed_mask(p))
    op = oracle.Problem.from_synth(p)
    before, after = op.evaluate(pop), op.evaluate(out)
    assert (before["flags"] != 0).sum() >= 6 and moves.sum() >= 4
    unit = 6.0 * 2.0 ** 30
    for c in range(16):
        drop = sum(c0[1] - cb[1] for m, v, sg, c0, cb, k in logs[c] if k is not None)
        assert after["severity"][c] <= before["severity"][c] + 1e-9
        np.testing.assert_allclose(before["severity"][c] - after["severity"][c], drop / unit,
                                   rtol=1e-9, atol=1e-12)
        if outcome[c] == R.NO_FOLD:
            assert before["flags"][c] == 0
            np.testing.assert_array_equal(out[c], pop[c])
        # pinned axes never move
        for m in range(2):
            moved = out[c, m] != pop[c, m]
            assert not np.any(moved & p.fixed_axes.T)
    # the magnitude and intensity of untouched candidates are unchanged
    same = moves == 0
    np.testing.assert_array_equal(after["obj"][same], before["obj"][same])
    # one pass clears most of the folds
    folded = before["flags"] != 0
    assert (after["flags"][folded] == 0).sum() >= folded.sum() // 2
