"""GPU parity of the elitist archive update and the multiplier adaptation
(Sec. 3, Sec. 4.3.2) through the C-ABI, bit for bit against the reference.

Sequences of updates on seeded offers: objective vectors on a small grid
(equal vectors, domination, ties), infeasible, folded and invalid offers,
NaN and infinite objectives; capacity pressure (points on a plane, all
non-dominated) with the box thinning at small and at the paper's capacity
(2000 members, 1,024 offers per update: 3,024 candidates); the steering
bound switched on part-way (members above it purged); the members' points
copied into their slots.  Every slot's objective vector and stamp, the
state, the best guidance value and the per-offer outputs must equal the
reference's."""
import math

import numpy as np
import pytest

from oracle import archive as ar

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def grid_offers(rs, n, grid):
    obj = rs.integers(0, grid, (n, 3)).astype(np.float32)
    flags = rs.choice(np.array([0, 0, 0, 0, 0, 1, 2, 4], np.uint8), n)
    sev = np.where(flags & 3, 0.5, 0.0).astype(np.float32)
    obj[rs.integers(0, n)] = [np.nan, 0, 0]
    obj[rs.integers(0, n)] = [0, -np.inf, 0]
    return obj, flags, sev


def plane_offers(rs, n):
    u = rs.random((n, 2))
    obj = np.stack([u[:, 0], u[:, 1], 2.0 - u[:, 0] - u[:, 1]], axis=1).astype(np.float32)
    return obj, np.zeros(n, np.uint8), np.zeros(n, np.float32)


def check(a, ref, ins, slot, ins_ref, slot_ref, what):
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.stamp.cpu().numpy(), ref.stamp.astype(np.int32), err_msg=f"stamps {what}")
    np.testing.assert_array_equal(a.obj.cpu().numpy(), ref.obj, err_msg=f"objectives {what}")
    st = a.state.cpu().numpy()
    assert st.tolist() == [len(ref.members()), ref.next_stamp, ref.levels, 0], (what, st)
    assert a.best.cpu().numpy()[0] == np.float32(ref.best_guidance()), what
    np.testing.assert_array_equal(ins.cpu().numpy(), ins_ref, err_msg=f"inserted {what}")
    np.testing.assert_array_equal(slot.cpu().numpy(), slot_ref.astype(np.int32), err_msg=f"slots {what}")


def run_sequence(cap, batches, bounds, n_points=0):
    a = morea.Archive(cap, n_points=n_points)
    ref = ar.Archive(cap)
    for k, ((obj, flags, sev), gmax) in enumerate(zip(batches, bounds)):
        out = dict(obj=dev(obj), flags=dev(flags), severity=dev(sev))
        pts = None
        if n_points:
            pts = dev(np.random.default_rng(k).normal(size=(len(flags), 2, 3, n_points)).astype(np.float32))
        ins, slot = a.update(out, pts=pts, guidance_max=gmax)
        ins_ref, slot_ref = ar.update(ref, obj, flags, sev, guidance_max=math.inf if gmax is None else gmax)
        check(a, ref, ins, slot, ins_ref, slot_ref, f"update {k}")
        if n_points:
            got = a.pts.cpu().numpy()
            want = pts.cpu().numpy()
            for i in np.flatnonzero(ins_ref):
                np.testing.assert_array_equal(got[slot_ref[i]], want[i])
    return a, ref


def test_grid_offers_sequence():
    rs = np.random.default_rng(1)
    batches = [grid_offers(rs, n, 5) for n in (37, 200, 1, 512, 64)]
    run_sequence(1000, batches, [None] * len(batches), n_points=7)


def test_capacity_thinning_small():
    rs = np.random.default_rng(2)
    batches = [plane_offers(rs, n) for n in (300, 300, 17, 300)]
    a, ref = run_sequence(40, batches, [None] * 4)
    assert ref.levels > 0


def test_capacity_thinning_paper_size():
    """2000 members and 1,024 offers per update (3,024 candidates)."""
    rs = np.random.default_rng(3)
    batches = [plane_offers(rs, 1024) for _ in range(3)]
    a, ref = run_sequence(2000, batches, [None] * 3)
    assert len(ref.members()) <= 2000 and ref.levels > 0


def test_steering_purge():
    """Guidance values spread over [0, 4]; the bound 1.5 s_G switches on at
    the third update and then follows the archive's best value."""
    rs = np.random.default_rng(4)
    a = morea.Archive(500)
    ref = ar.Archive(500)
    for k in range(6):
        obj, flags, sev = plane_offers(rs, 256)
        obj[:, 2] = (rs.random(256) * 4.0 * (0.8 ** k)).astype(np.float32)
        gmax = None if k < 2 else ar.steering_bound(ref.best_guidance())
        if gmax is not None:
            assert gmax == float(np.float32(1.5) * a.best.cpu().numpy()[0])
        out = dict(obj=dev(obj), flags=dev(flags), severity=dev(sev))
        ins, slot = a.update(out, guidance_max=gmax)
        ins_ref, slot_ref = ar.update(ref, obj, flags, sev, guidance_max=math.inf if gmax is None else gmax)
        check(a, ref, ins, slot, ins_ref, slot_ref, f"steering update {k}")
    assert ref.best_guidance() < 0.2


def test_clear_and_empty_update():
    a = morea.Archive(16)
    ref = ar.Archive(16)
    out = dict(obj=dev(np.zeros((0, 3), np.float32)), flags=dev(np.zeros(0, np.uint8)),
               severity=dev(np.zeros(0, np.float32)))
    ins, slot = a.update(out)
    torch.cuda.synchronize()
    assert a.state.cpu().numpy().tolist() == [0, 0, 0, 0]
    assert math.isinf(a.best.cpu().numpy()[0])
    rs = np.random.default_rng(5)
    obj, flags, sev = grid_offers(rs, 30, 4)
    ins, slot = a.update(dict(obj=dev(obj), flags=dev(flags), severity=dev(sev)))
    ins_ref, slot_ref = ar.update(ref, obj, flags, sev)
    check(a, ref, ins, slot, ins_ref, slot_ref, "after clear")
    a.clear()
    torch.cuda.synchronize()
    assert np.all(a.stamp.cpu().numpy() == -1) and np.all(np.isinf(a.obj.cpu().numpy()))


def test_argument_errors():
    lib = morea.load_library()
    a = morea.Archive(3000)
    obj = dev(np.zeros((1100, 3), np.float32))
    fl = dev(np.zeros(1100, np.uint8))
    sv = dev(np.zeros(1100, np.float32))
    ins = torch.empty(1100, dtype=torch.uint8, device="cuda")
    slot = torch.empty(1100, dtype=torch.int32, device="cuda")
    P = morea._dev_ptr
    for n, cap, g in ((1100, 100, 1.0), (1024, 3100, 1.0), (10, 100, float("nan")), (10, 0, 1.0)):
        st = lib.morea_archive_update(n, P(obj), P(fl), P(sv), None, 0, g, cap, P(a.obj), P(a.stamp), None,
                                      P(a.state), P(a.best), P(ins), P(slot), None)
        assert st in (morea.MOREA_EINVAL, morea.MOREA_ERANGE), (n, cap, g, st)
    assert lib.morea_archive_clear(5000, P(a.obj), P(a.stamp), P(a.state), P(a.best), None) == morea.MOREA_EINVAL


def test_mark_and_adapt_multipliers():
    rs = np.random.default_rng(6)
    k, G, n_par, n_ev = 5, 40, 30, 3000
    ep = rs.integers(-1, n_par + 1, n_ev).astype(np.int32)
    eg = rs.integers(-1, G + 1, n_ev).astype(np.int32)
    ec = rs.integers(-1, k + 1, n_ev).astype(np.int32)
    acc = (rs.random(n_ev) < 0.1).astype(np.uint8)
    pin = (rs.random(n_par) < 0.5).astype(np.uint8)
    mult = rs.choice(np.array([0.5, 0.9, 1.0, 1.5, 9.9], np.float32), (k, G))
    nis = rs.integers(0, 30, (k, G)).astype(np.int32)
    imp = np.zeros((k, G), np.uint8)
    d_imp, d_mult, d_nis = dev(imp), dev(mult), dev(nis)
    morea.morea_mark_improvements(dev(ep), dev(eg), dev(ec), dev(acc), dev(pin), d_imp)
    torch.cuda.synchronize()
    ar.mark_improvements(imp, ep, eg, ec, acc, pin)
    np.testing.assert_array_equal(d_imp.cpu().numpy(), imp)
    assert 0 < imp.sum() < imp.size
    nis64 = nis.astype(np.int64)
    morea.morea_adapt_multipliers(d_imp, d_mult, d_nis)
    torch.cuda.synchronize()
    ar.adapt_multipliers(imp, mult, nis64)
    np.testing.assert_array_equal(d_mult.cpu().numpy(), mult)
    np.testing.assert_array_equal(d_nis.cpu().numpy(), nis64.astype(np.int32))
    assert not d_imp.cpu().numpy().any()
