"""GPU parity of the selection and clustering at the start of a generation
(Sec. 3) through the C-ABI: on seeded objective vectors, flags and
severities the selection, its size, the cluster offsets and members and
every solution's cluster equal the reference exactly (fronts by peeling,
index tie rules, FP64 normalised distances); ties, infeasible and invalid
solutions, a steering bound, fewer selected solutions than clusters, and a
full block of 1,024 solutions are covered."""
import numpy as np
import pytest

from oracle import selection as sl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def run(obj, flags, sev, size, k, gmax=None):
    out = dict(obj=torch.from_numpy(np.ascontiguousarray(obj, np.float32)).cuda(),
               flags=torch.from_numpy(np.ascontiguousarray(flags, np.uint8)).cuda(),
               severity=torch.from_numpy(np.ascontiguousarray(sev, np.float32)).cuda())
    res = morea.select_clusters(out, size, k, guidance_max=gmax)
    torch.cuda.synchronize()
    return {kk: v.cpu().numpy() for kk, v in res.items()}


def check(obj, flags, sev, size, k, gmax=None):
    got = run(obj, flags, sev, size, k, gmax)
    sel, leaders, members, cluster_of = sl.clusters(obj, flags, sev, size, k,
                                                    float("inf") if gmax is None else float(np.float32(gmax)))
    n_sel = int(got["n_selected"][0])
    assert n_sel == len(sel)
    assert got["selection"][:n_sel].tolist() == sel
    off = got["clu_off"]
    assert off[0] == 0 and len(off) == k + 1
    for j in range(k):
        assert got["clu_members"][off[j]:off[j + 1]].tolist() == members[j], j
    assert got["cluster_of"].tolist() == cluster_of
    return n_sel, leaders


def test_hand_worked_one_dimensional():
    xs = [0.0, 1.0, 2.0, 3.0, 10.0, 4.0, 9.0]
    obj = np.array([(x, 0, 0) for x in xs], np.float32)
    check(obj, np.zeros(7, np.uint8), np.zeros(7, np.float32), 7, 3)


def test_random_mixed_feasibility():
    rs = np.random.default_rng(21)
    n = 60
    obj = rs.normal(size=(n, 3)).astype(np.float32)
    fl = rs.choice(np.array([0, 0, 0, 0, 1, 2, 4], np.uint8), n)
    sv = rs.uniform(0, 1, n).astype(np.float32)
    obj[5, 1] = np.nan
    for size, k in ((30, 5), (60, 10), (3, 5), (0, 2)):
        print("case", size, k, flush=True)
        if size == 0:
            got = run(obj, fl, sv, 0, 2)
            assert got["n_selected"][0] == 0 and np.all(got["cluster_of"] == -1)
            continue
        check(obj, fl, sv, size, k)


def test_grid_ties_and_steering():
    rs = np.random.default_rng(22)
    n = 300
    obj = rs.integers(0, 4, (n, 3)).astype(np.float32)
    obj[:, 2] *= np.float32(0.5)
    fl = rs.choice(np.array([0, 0, 0, 1, 2, 3], np.uint8), n)
    sv = (rs.integers(0, 3, n) * 0.5).astype(np.float32)
    n_sel, leaders = check(obj, fl, sv, 105, 10)
    assert n_sel == 105
    check(obj, fl, sv, 105, 10, gmax=0.75)


def test_infinite_objectives_are_invalid():
    """Regression: an infinite objective once passed as valid, normalised to
    NaN and let a solution join every cluster past its m slots.  Now such
    solutions are invalid (never selected, cluster -1), on a case whose
    clusters fill members_cap exactly."""
    rs = np.random.default_rng(24)
    n = 40
    obj = rs.normal(size=(n, 3)).astype(np.float32)
    fl = np.zeros(n, np.uint8)
    sv = np.zeros(n, np.float32)
    obj[3, 0] = np.inf
    obj[7, 1] = -np.inf
    obj[11, 2] = np.inf
    sv[13] = np.inf
    for size, k in ((20, 4), (36, 6), (40, 5)):
        print("case", size, k, flush=True)
        n_sel, _ = check(obj, fl, sv, size, k)
        got = run(obj, fl, sv, size, k)
        m = min(n_sel, -(-2 * n_sel // k))
        assert got["clu_off"][k] == min(k, n_sel) * m <= len(got["clu_members"])
        if size < 40:
            assert got["clu_off"][k] == len(got["clu_members"])      # the clusters fill members_cap
        for i in (3, 7, 11, 13):
            assert got["cluster_of"][i] == -1 and i not in got["selection"][:n_sel]


def test_full_block():
    rs = np.random.default_rng(23)
    n = 1024
    obj = rs.normal(size=(n, 3)).astype(np.float32)
    fl = rs.choice(np.array([0, 0, 0, 0, 0, 1], np.uint8), n)
    sv = rs.uniform(0, 1, n).astype(np.float32)
    check(obj, fl, sv, 40, 4)
    with pytest.raises(morea.MoreaError):
        run(np.zeros((1025, 3), np.float32), np.zeros(1025, np.uint8), np.zeros(1025, np.float32), 10, 2)


def test_argument_errors():
    """Host-side validation of the selection, sampling and acceptance calls."""
    import ctypes
    L = morea.load_library()
    dev_f = torch.zeros(12, dtype=torch.float32, device="cuda")
    dev_u8 = torch.zeros(4, dtype=torch.uint8, device="cuda")
    dev_i = torch.zeros(64, dtype=torch.int32, device="cuda")
    P = ctypes.c_void_p
    args = [P(dev_f.data_ptr()), P(dev_u8.data_ptr()), P(dev_f.data_ptr()), 4, 4, 2, float("inf"),
            P(dev_i.data_ptr()), P(dev_i.data_ptr()), P(dev_i.data_ptr()), P(dev_i.data_ptr())]
    # members_cap below k * ceil(2 min(size, n) / k) = 8
    assert L.morea_select_clusters(*args, 7, P(dev_i.data_ptr()), None) == morea.MOREA_ERANGE
    assert L.morea_select_clusters(*args[:6], float("nan"), *args[7:], 8, P(dev_i.data_ptr()), None) == \
        morea.MOREA_EINVAL
    assert L.morea_select_clusters(*args[:4], -1, *args[5:], 8, P(dev_i.data_ptr()), None) == morea.MOREA_EINVAL
    torch.cuda.synchronize()
