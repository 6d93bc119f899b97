"""GPU tests of the learned pre-screen: matrix-core forward pass against an
FP64 reference with the same BF16 rounding points, gradients against the FP64
oracle's backpropagation, training, selection, and what the trained network
gains over random pre-selection at the same exact-evaluation budget."""
import numpy as np
import pytest

import synth
from conftest import oracle_problem, synth_problem
import oracle
from oracle import mlp, surrogate_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def mixed_forward(theta, X):
    """FP64 forward with the kernel's rounding points: BF16 inputs, W1, W2
    and layer-1 activations; FP32 biases and output layer."""
    p = mlp.unpack(theta)
    z1 = mlp.bf16(X) @ mlp.bf16(p["W1"]).T + p["b1"]
    h1 = mlp.bf16(np.maximum(z1, 0.0))
    z2 = h1 @ mlp.bf16(p["W2"]).T + p["b2"]
    return np.maximum(z2, 0.0) @ p["w3"] + p["b3"][0]


def random_theta(seed, scale=1.0):
    rs = np.random.default_rng(seed)
    p = {}
    for name, shape in mlp.SHAPES:
        fan = shape[1] if len(shape) == 2 else 1
        p[name] = rs.normal(0, scale * np.sqrt(2.0 / fan) if len(shape) == 2 else 0.1, shape)
    return mlp.pack(p).astype(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def c1_surrogate():
    p = synth_problem(1)
    prob = morea.Problem.from_synth(p, max_population=16)
    return p, prob, morea.Surrogate(prob, max_rows=8192, seed=3)


def test_forward_matches_reference(c1_surrogate):
    _, _, s = c1_surrogate
    theta = random_theta(1)
    s.set_params(theta)
    rs = np.random.default_rng(2)
    X = rs.normal(0, 1, (1000, mlp.N_IN)).astype(np.float32)        # 1000: ragged last tile
    y = s.predict_rows(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = mixed_forward(theta, X.astype(np.float64))
    assert np.max(np.abs(y - ref)) <= 1e-3 * (np.std(ref) + 1e-3)
    pure, _ = mlp.forward(theta, X)
    assert np.corrcoef(y, pure)[0, 1] > 0.999


def test_gradients_match_oracle(c1_surrogate):
    """Every gradient entry against the FP64 backpropagation with the
    kernels' BF16 rounding points (inputs, W1, W2, h1, and the two
    back-propagated activations dz2 and dz1 fed to the matrix cores).

    Bound per entry: FP32 accumulation over the 777 rows (1e-4 of the
    entry's L1 mass, the sum of |term| over rows) plus two BF16 rounding
    flips of single terms where the GPU's FP32 value and the reference's FP64
    value straddle a rounding boundary (2^-7 of the largest |term|)."""
    _, _, s = c1_surrogate
    theta = random_theta(4)
    s.set_params(theta)
    rs = np.random.default_rng(5)
    X = rs.normal(0, 1, (777, mlp.N_IN)).astype(np.float32)
    t = rs.normal(0, 1, 777).astype(np.float32)
    g, loss = s.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda())
    g = g.cpu().numpy().astype(np.float64)
    ref = mlp.gradient(theta, X, t, rnd=mlp.bf16)
    lref = mlp.loss(theta, X, t, rnd=mlp.bf16)
    assert abs(loss.item() - lref) <= 1e-5 * lref
    # per-entry term masses from the same forward/backward quantities
    rb = mlp.bf16
    p = mlp.unpack(theta)
    y, (Xb, z1, h1, z2, h2) = mlp.forward(theta, X, rb)
    dy = 2.0 * (y - t) / len(t)
    dz2 = np.outer(dy, p["w3"]) * (z2 > 0)
    dz2b = rb(dz2)
    dz1 = (dz2b @ rb(p["W2"])) * (h1 > 0)
    dz1b = rb(dz1)
    mass = {"W1": (np.abs(dz1b).T @ np.abs(Xb), np.abs(dz1b).max(0)[:, None] * np.abs(Xb).max(0)[None]),
            "b1": (np.abs(dz1).sum(0), np.abs(dz1).max(0)),
            "W2": (np.abs(dz2b).T @ np.abs(h1), np.abs(dz2b).max(0)[:, None] * np.abs(h1).max(0)[None]),
            "b2": (np.abs(dz2).sum(0), np.abs(dz2).max(0)),
            "w3": (np.abs(h2).T @ np.abs(dy), np.abs(h2).max(0) * np.abs(dy).max()),
            "b3": (np.array([np.abs(dy).sum()]), np.array([np.abs(dy).max()]))}
    o = 0
    for name, shape in mlp.SHAPES:
        n = int(np.prod(shape))
        a, b = g[o:o + n], ref[o:o + n]
        o += n
        l1, big = (m.reshape(-1) for m in mass[name])
        tol = 1e-4 * l1 + 2.0 ** -7 * big + 1e-12
        bad = np.abs(a - b) > tol
        assert not bad.any(), (name, int(np.argmax(bad)), a[bad][:3], b[bad][:3])
        assert np.linalg.norm(a - b) <= 2e-3 * np.linalg.norm(b), name


def test_gradients_finite_differences_on_gpu(c1_surrogate):
    """Central differences of the GPU's own loss for parameters downstream of
    every BF16 rounding (b3, w3, b2; the loss is smooth in them away from
    ReLU kinks): the GPU gradient is the derivative of the GPU loss."""
    _, _, s = c1_surrogate
    theta = random_theta(12)
    rs = np.random.default_rng(13)
    X = torch.from_numpy(rs.normal(0, 1, (512, mlp.N_IN)).astype(np.float32)).cuda()
    t = torch.from_numpy(rs.normal(0, 1, 512).astype(np.float32)).cuda()
    s.set_params(theta)
    g, _ = s.gradients(X, t)
    g = g.cpu().numpy().astype(np.float64)
    offs = {}
    o = 0
    for name, shape in mlp.SHAPES:
        offs[name] = o
        o += int(np.prod(shape))
    picks = [offs["b3"], offs["w3"] + 3, offs["w3"] + 77, offs["b2"] + 5, offs["b2"] + 100]
    eps = 1e-2
    for i in picks:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        s.set_params(tp)
        _, lp = s.gradients(X, t)
        s.set_params(tm)
        _, lm = s.gradients(X, t)
        fd = (lp.item() - lm.item()) / (2 * eps)
        assert abs(fd - g[i]) <= 2e-2 * abs(g[i]) + 2e-4, (i, fd, g[i])
    s.set_params(theta)


def family(p, prob, n_parents=2, per_parent=8, seed=None):
    """Parents and offspring (synth.make_offspring), both evaluated in full:
    (parents, offspring, parent_of, parent cache, offspring cache) on the
    GPU."""
    par, off = synth.make_offspring(p, n_parents=n_parents, per_parent=per_parent, seed=seed)
    dp, do = torch.from_numpy(par).cuda(), torch.from_numpy(off).cuda()
    of = torch.arange(n_parents, dtype=torch.int32, device="cuda").repeat_interleave(per_parent)
    pc, oc = prob.new_cache(len(par)), prob.new_cache(len(off))
    prob.eval_full(dp, cache=pc)
    prob.eval_full(do, cache=oc)
    return dp, do, of, pc, oc


def test_training_reduces_loss(c1_surrogate):
    p, prob, s = c1_surrogate
    s.set_params(random_theta(7, scale=0.5))
    dp, do, of, pc, oc = family(p, prob)
    X = s.features(do, dp, pc, of).reshape(-1, s.n_features).contiguous()
    t = s.targets(oc, len(do), pc, len(dp), of).reshape(-1).contiguous()
    loss = torch.empty(1, device="cuda")
    losses = []
    for step in range(300):
        s.train_step(X, t, 2e-3, loss_out=loss)
        if step % 50 == 0 or step == 299:
            losses.append(loss.item())
    assert losses[-1] < 0.5 * losses[0], losses


def test_features_and_stats(c1_surrogate):
    """Every input row against the FP64 reference (oracle surrogate_inputs),
    one offspring moved far outside the image box (clamped samples): the
    moves within FP32 subtraction, the estimated changes within FP32
    arithmetic on h values of at most the image range squared (1e-5 of it,
    over h_scale, plus 1e-4 relative), the parent's terms within the records'
    parity bar; h_scale to FP32 summation; the statistics are the library's
    own, checked against the reference by check_stats."""
    p, prob, s = c1_surrogate
    assert s.n_features == mlp.N_IN == 23
    dp, do, of, pc, oc = family(p, prob, seed=41)
    off = do.cpu().numpy()
    off[0, 1] += np.float32(3.0 * max(p.dims))
    F = s.features(torch.from_numpy(off).cuda(), dp, pc, of).cpu().numpy().astype(np.float64)
    st, cnt = s.stats()
    op = oracle_problem(1)
    hs = surrogate_inputs.h_scale(op)
    np.testing.assert_allclose(s.h_scale, hs, rtol=1e-5)
    ref_st, _ = surrogate_inputs.region_stats(op)
    par = dp.cpu().numpy()
    prec = op.evaluate(par, records=True)["records"]
    want = surrogate_inputs.features(op, ref_st, off, par, prec, of.cpu().numpy())
    scale2 = float(np.abs(p.image_tgt).max()) ** 2
    np.testing.assert_allclose(F[..., :12], want[..., :12], rtol=0, atol=1e-5)
    np.testing.assert_allclose(F[..., 12:15], want[..., 12:15], rtol=1e-4, atol=1e-5 * scale2 / hs)
    np.testing.assert_array_equal(F[..., 15:21], np.broadcast_to(st[:, :6], F[..., 15:21].shape))
    np.testing.assert_allclose(F[..., 21], np.broadcast_to(st[:, 6] / s.h_scale, F[..., 21].shape), rtol=1e-6)
    np.testing.assert_allclose(F[..., 22], want[..., 22], rtol=1e-5, atol=2e-6 * scale2 / hs)
    assert np.isfinite(F).all()
    # an offspring whose parent index is out of range gets a row of NaN
    bad_of = torch.tensor([0, len(par)], dtype=torch.int32, device="cuda")
    Fo = s.features(do[:2].contiguous(), dp, pc, bad_of).cpu().numpy()
    Fg = s.features(do[:2].contiguous(), dp, pc, of[:2].contiguous()).cpu().numpy()
    np.testing.assert_array_equal(Fo[0], Fg[0])
    assert np.all(np.isnan(Fo[1]))
    V = int(np.prod(p.dims))
    assert cnt.sum() == V            # the reference mesh tiles the grid exactly
    check_stats(st, cnt, op)


def check_stats(st, cnt, op):
    """The 8 region statistics against the FP64 reference element by element:
    counts exact; means, fractions and the count ratio within FP32 summation
    of at most a few thousand values (1e-5 relative); standard deviations
    within the bound that the FP32 variance E[x^2] - E[x]^2 carries,
    4 n 2^-24 E[x^2], divided by the sum of the two deviations."""
    ref, rcnt = surrogate_inputs.region_stats(op)
    np.testing.assert_array_equal(cnt, rcnt)
    st = st.astype(np.float64)
    for k in (0, 2, 3, 5, 6, 7):
        np.testing.assert_allclose(st[:, k], ref[:, k], rtol=1e-5, atol=1e-7, err_msg=f"stat {k}")
    n = np.maximum(rcnt, 1).astype(np.float64)
    for k, mean in ((1, 0), (4, 3)):
        ex2 = ref[:, k] ** 2 + ref[:, mean] ** 2
        ev = 4.0 * n * 2.0 ** -24 * ex2 + 1e-12
        tol = ev / np.maximum(st[:, k] + ref[:, k], np.sqrt(ev))
        bad = np.abs(st[:, k] - ref[:, k]) > tol
        assert not bad.any(), (k, np.argwhere(bad)[:3].ravel(), st[bad, k][:3], ref[bad, k][:3])


def test_stats_quantized_storage():
    """The statistics of a BF16 problem read the stored (rounded) images."""
    p = synth_problem(1)
    prob = morea.Problem.from_synth(p, storage="bf16", max_population=1)
    s = morea.Surrogate(prob, max_rows=1024, seed=1)
    st, cnt = s.stats()
    op = oracle.Problem.from_synth(p, image_src=oracle.quantize(p.image_src, "bf16"),
                                   image_tgt=oracle.quantize(p.image_tgt, "bf16"))
    check_stats(st, cnt, op)


def test_targets_match_oracle_records(c1_surrogate):
    """Training targets, the offspring's (h_S + h_T) / (n_S + n_T) per tet
    minus its parent's over h_scale, from the full evaluations' caches against
    the oracle's per-tet records: twice the records' bound (1e-6 per sample
    plus 2e-6 relative) divided by the samples, over h_scale; NaN rows for a
    parent index out of range."""
    p, prob, s = c1_surrogate
    dp, do, of, pc, oc = family(p, prob, seed=31)
    t = s.targets(oc, len(do), pc, len(dp), of).cpu().numpy().astype(np.float64)
    op = oracle_problem(1)
    hs = surrogate_inputs.h_scale(op)
    want = surrogate_inputs.targets(op.evaluate(do.cpu().numpy(), records=True)["records"],
                                    op.evaluate(dp.cpu().numpy(), records=True)["records"], of.cpu().numpy(), hs)
    np.testing.assert_allclose(t, want, rtol=6e-6, atol=3e-6 / hs)
    assert (np.abs(want) > 0).mean() > 0.3
    bad = of.clone()
    bad[3] = -1
    t2 = s.targets(oc, len(do), pc, len(dp), bad).cpu().numpy()
    assert np.all(np.isnan(t2[3]))
    np.testing.assert_array_equal(np.delete(t2, 3, axis=0), np.delete(t.astype(np.float32), 3, axis=0))


def test_select_and_gather():
    rs = np.random.default_rng(8)
    score = rs.normal(size=3000).astype(np.float32)
    score[10] = score[20]                                 # a tie: lower index first
    pts = torch.from_numpy(rs.normal(size=(3000, 2, 3, 5)).astype(np.float32)).cuda()
    idx, sel = morea.morea_surrogate_select(torch.from_numpy(score).cuda(), 257, pts)
    want = np.argsort(score, kind="stable")[:257]
    np.testing.assert_array_equal(idx.cpu().numpy(), want)
    np.testing.assert_array_equal(sel.cpu().numpy(), pts.cpu().numpy()[want])


def test_prescreen_equals_weighted_row_predictions(c1_surrogate):
    """The fused pre-screen's score is sum_tet w_tet (parent term + h_scale
    row prediction) / sum_tet w_tet over the same rows built explicitly, w_tet
    the offspring's source plus target |volume| of the tet (the reference's
    score form); an offspring without a valid parent scores +inf."""
    p, prob, s = c1_surrogate
    s.set_params(random_theta(9, scale=0.5))
    dp, do, of, pc, oc = family(p, prob, seed=43)
    score = s.prescreen(do, dp, pc, of).cpu().numpy()
    F = s.features(do, dp, pc, of)
    y = s.predict_rows(F.reshape(-1, s.n_features).contiguous()).cpu().numpy().astype(np.float64)
    y = y.reshape(len(do), -1)
    op = oracle_problem(1)
    prec = op.evaluate(dp.cpu().numpy(), records=True)["records"]
    want = surrogate_inputs.score(op, do.cpu().numpy(), prec, of.cpu().numpy(), y * s.h_scale / surrogate_inputs.h_scale(op))
    np.testing.assert_allclose(score, want, rtol=1e-4, atol=1e-6)
    bad = of.clone()
    bad[5] = len(dp)
    score2 = s.prescreen(do, dp, pc, bad).cpu().numpy()
    assert score2[5] == np.inf
    np.testing.assert_array_equal(np.delete(score2, 5), np.delete(score, 5))


def test_prescreen_workspace_regrows_and_orders_do_not_matter(c1_surrogate):
    """Two pre-screens in a row, the second with more parents (the workspace
    grows) and the offspring in another order, and a third with fewer: each
    score equals the offspring's score in a fresh single-family call."""
    p, prob, s = c1_surrogate
    s.set_params(random_theta(21, scale=0.5))
    dp, do, of, pc, _ = family(p, prob, n_parents=2, per_parent=8, seed=51)
    s1 = s.prescreen(do, dp, pc, of).cpu().numpy()
    # four parents: the two above plus two more, offspring reversed
    dp2, do2, of2, pc2, _ = family(p, prob, n_parents=2, per_parent=8, seed=52)
    par4 = torch.cat([dp2, dp]).contiguous()
    pc4 = prob.new_cache(4)
    prob.eval_full(par4, cache=pc4)
    rev = torch.arange(15, -1, -1, device="cuda")
    s2 = s.prescreen(do[rev].contiguous(), par4, pc4, (of[rev] + 2).to(torch.int32).contiguous()).cpu().numpy()
    np.testing.assert_allclose(s2, s1[::-1], rtol=1e-6, atol=1e-9)
    s3 = s.prescreen(do[:3].contiguous(), dp, pc, of[:3].contiguous()).cpu().numpy()
    np.testing.assert_allclose(s3, s1[:3], rtol=1e-6, atol=1e-9)


def test_features_bf16_storage_read_the_stored_images():
    """A BF16 problem's features sample the stored (rounded) images: against
    the reference on the quantized images."""
    p = synth_problem(1)
    prob = morea.Problem.from_synth(p, storage="bf16", max_population=16)
    s = morea.Surrogate(prob, max_rows=1024, seed=2)
    dp, do, of, pc, _ = family(p, prob, n_parents=1, per_parent=4, seed=61)
    F = s.features(do, dp, pc, of).cpu().numpy().astype(np.float64)
    op = oracle.Problem.from_synth(p, image_src=oracle.quantize(p.image_src, "bf16"),
                                   image_tgt=oracle.quantize(p.image_tgt, "bf16"))
    st, _ = surrogate_inputs.region_stats(op)
    hs = surrogate_inputs.h_scale(op)
    np.testing.assert_allclose(s.h_scale, hs, rtol=1e-5)
    prec = op.evaluate(dp.cpu().numpy(), records=True)["records"]
    want = surrogate_inputs.features(op, st, do.cpu().numpy(), dp.cpu().numpy(), prec, of.cpu().numpy())
    scale2 = float(np.abs(p.image_tgt).max()) ** 2
    np.testing.assert_allclose(F[..., 12:15], want[..., 12:15], rtol=1e-4, atol=1e-5 * scale2 / hs)
    np.testing.assert_allclose(F[..., 22], want[..., 22], rtol=1e-5, atol=2e-6 * scale2 / hs)


def spearman(a, b):
    ra = np.argsort(np.argsort(a))
    rb = np.argsort(np.argsort(b))
    return np.corrcoef(ra, rb)[0, 1]


def test_surrogate_gain_config5():
    """Offspring of 512 parents, 8 each (source fixed, the parents evaluated
    exactly), exact budget 512 of the 4,096.  Trained on ~1 M exact per-tet
    changes of 37 other families, the surrogate's ranking, on three batches
    drawn with different seeds, must correlate with the exact f_int (Spearman
    rho >= 0.5), its 512 must close at least half of the gap between the
    batch mean (the expected value of a random 512) and the true best 512, and
    it must beat ranking by the parent's exact f_int alone."""
    p = synth_problem(5)
    prob = morea.Problem.from_synth(p, max_population=4096)
    s = morea.Surrogate(prob, max_rows=8192, seed=11)
    dp, do, of, pc, oc = family(p, prob, n_parents=37, per_parent=8, seed=105)
    X = s.features(do, dp, pc, of).reshape(-1, s.n_features).contiguous()
    t = s.targets(oc, len(do), pc, len(dp), of).reshape(-1).contiguous()
    n = t.numel()
    assert n > 1_000_000
    g = torch.Generator(device="cpu").manual_seed(0)
    for epoch in range(10):
        perm = torch.randperm(n, generator=g).cuda()
        for b in range(0, n - 8191, 8192):
            sel = perm[b:b + 8192]
            s.train_step(X[sel].contiguous(), t[sel].contiguous(), 2e-3 if epoch < 6 else 5e-4)
    del X, t, oc
    prob512 = morea.Problem.from_synth(p, max_population=512)
    for seed in (5, 205, 305):
        dp, do, of, pc, _ = family(p, prob, n_parents=512, per_parent=8, seed=seed)
        f = prob.eval_full(do)["obj"][:, 0].cpu().numpy().astype(np.float64)
        fp = prob.eval_full(dp)["obj"][:, 0].cpu().numpy().astype(np.float64)
        score = s.prescreen(do, dp, pc, of)
        idx, chosen = morea.morea_surrogate_select(score, 512, do)
        idx = idx.cpu().numpy()
        f_sel = prob512.eval_full(chosen)["obj"][:, 0].cpu().numpy()
        np.testing.assert_allclose(f_sel, f[idx], rtol=1e-6)
        best = np.argsort(f)[:512]
        by_parent = np.argsort(fp[of.cpu().numpy()], kind="stable")[:512]
        m_sur, m_all, m_best, m_par = f[idx].mean(), f.mean(), f[best].mean(), f[by_parent].mean()
        rho = spearman(score.cpu().numpy(), f)
        gap = (m_all - m_sur) / (m_all - m_best)
        print(f"seed {seed}: surrogate {m_sur:.6f} batch mean {m_all:.6f} best {m_best:.6f} "
              f"parent-only {m_par:.6f} rho {rho:.3f} gap closed {gap:.3f}", flush=True)
        assert rho >= 0.5
        assert gap >= 0.5
        assert m_sur < m_par
