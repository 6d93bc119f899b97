"""GPU parity of reduced-precision image storage (BF16 / FP16, FP32 arithmetic).

The parity reference is the oracle run on the same quantized images (the
stored values, exactly upcast): counts and flags bit-exact, objectives within
1e-5.  The effect of the storage itself (against the FP32-image oracle) is
measured and bounded separately: it is a property of the data, not an error
of the evaluator."""
import numpy as np
import pytest

import oracle
import synth
from conftest import synth_problem
from parity import assert_parity, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def quantized_oracle(p, storage):
    return oracle.Problem.from_synth(p, image_src=oracle.quantize(p.image_src, storage),
                                     image_tgt=oracle.quantize(p.image_tgt, storage))


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_c1_reduced_storage(storage):
    p = synth_problem(1)
    pop = synth.make_population(p, perturb_source=True, fold_fraction=0.25)
    prob = morea.Problem.from_synth(p, storage=storage, max_population=len(pop))
    g = to_host(prob.eval_full(torch.from_numpy(pop).cuda()))
    assert_parity(g, quantized_oracle(p, storage).evaluate(pop), what=storage)
    # storage effect against FP32 images: small but not zero
    o32 = oracle.Problem.from_synth(p).evaluate(pop)
    eff = np.abs(g["obj"][:, 0] - o32["obj"][:, 0]) / o32["obj"][:, 0]
    assert eff.max() < 5e-2


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_c4_full_size_sampled(storage):
    """192x192x128, 9,126 tets, population 256 in one launch; two candidates
    against the oracle on the quantized images."""
    p = synth_problem(4)
    pop = synth.make_population(p)
    prob = morea.Problem.from_synth(p, storage=storage, max_population=len(pop))
    g = to_host(prob.eval_full(torch.from_numpy(pop).cuda()))
    V = int(np.prod(p.dims))
    free = g["flags"] == 0
    assert np.all(g["counts"][free] == V)
    idx = [0, 129]
    assert_parity(g, quantized_oracle(p, storage).evaluate(pop[idx]), idx=idx, what=storage)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_c4_partial(storage):
    """192x192x128, 16 parents x 8 groups of 4-48 points: the partial
    evaluations equal a full evaluation of each child with the same storage
    (counts and flags exact, objectives within 1e-5) and the oracle on the
    quantized images for three children."""
    p = synth_problem(4)
    parents = synth.make_population(p, pop=16)
    off, pts = synth.make_groups(p, n_groups=8, sizes=(4, 48))
    ep, eg, new = synth.make_children(p, parents, off, pts)
    prob = morea.Problem.from_synth(p, storage=storage, max_population=16)
    prob.set_groups(off, pts)
    prob.reserve_partial(len(ep))
    dpar = torch.from_numpy(parents).cuda()
    cache = prob.new_cache(16)
    prob.eval_full(dpar, cache=cache)
    g = to_host(prob.eval_partial(dpar, cache, torch.from_numpy(ep).cuda(), torch.from_numpy(eg).cuda(),
                                  torch.from_numpy(new).cuda()))
    kids = np.stack([synth.apply_child(parents, off, pts, ep, eg, new, e) for e in range(len(ep))])
    full = to_host(morea.Problem.from_synth(p, storage=storage, max_population=len(kids)).eval_full(
        torch.from_numpy(kids).cuda()))
    np.testing.assert_array_equal(full["counts"], g["counts"])
    np.testing.assert_array_equal(full["flags"], g["flags"])
    rel = np.abs(full["obj"].astype(np.float64) - g["obj"]) / np.abs(full["obj"])
    assert rel.max() < 1e-5
    few = [0, 37, 101]
    assert_parity(g, quantized_oracle(p, storage).evaluate(kids[few]), idx=few, what=f"c4 partial {storage}")
    # the other launch form gives the same outputs bit for bit
    shape = prob.partial_shape()
    prob.set_partial_shape(*((0, 0) if shape != (0, 0) else (256, 8)))
    g2 = to_host(prob.eval_partial(dpar, cache, torch.from_numpy(ep).cuda(), torch.from_numpy(eg).cuda(),
                                   torch.from_numpy(new).cuda()))
    for k in g:
        np.testing.assert_array_equal(g2[k], g[k], err_msg=f"launch forms {k}")
