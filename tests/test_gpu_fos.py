"""GPU check of one generation's colour-batched partial evaluations: the
library's FOS elements (set-cover edges, Sec. 4.2.1) registered as groups, one
morea_eval_partial call per DSATUR colour over every (solution, element of the
colour) child, each against the oracle's full evaluation of the child."""
import numpy as np
import pytest

import synth
from conftest import oracle_problem, synth_problem
from parity import assert_parity, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def test_c1_generation_sweep():
    p = synth_problem(1)
    pop = synth.make_population(p, pop=4, seed=61, perturb_source=True, fold_fraction=0.0)
    elements, colors, n_colors = morea.build_fos(p.n_points, p.tets)
    assert n_colors >= 2 and len(elements) >= p.n_points // 2
    prob = morea.Problem.from_synth(p, max_population=4)
    prob.set_groups(np.arange(0, 2 * len(elements) + 1, 2, dtype=np.int32), elements.reshape(-1))
    per = [np.flatnonzero(colors == c).astype(np.int32) for c in range(n_colors)]
    prob.reserve_partial(4 * max(len(g) for g in per))
    par = torch.from_numpy(pop).cuda()
    cache = prob.new_cache(4)
    prob.eval_full(par, cache=cache)
    rs = np.random.default_rng(2)
    for c, g in enumerate(per):
        ep = np.repeat(np.arange(4, dtype=np.int32), len(g))
        eg = np.tile(g, 4)
        pts = elements[eg]
        new = pop[ep[:, None, None, None], np.arange(2)[None, None, :, None], np.arange(3)[None, None, None, :],
                  pts[:, :, None, None]].astype(np.float64)
        new = (new + rs.normal(0, 0.5, new.shape) * ~p.fixed_axes[pts][:, :, None, :]).astype(np.float32)
        out = prob.eval_partial(par, cache, torch.from_numpy(ep).cuda(), torch.from_numpy(eg).cuda(),
                                torch.from_numpy(new.reshape(-1, 2, 3)).cuda())
        g_out = to_host(out)
        sel = rs.choice(len(ep), min(6, len(ep)), replace=False)
        kids = []
        for e in sel:
            child = pop[ep[e]].copy()
            child[:, :, elements[eg[e]]] = new[e].transpose(1, 2, 0)
            kids.append(child)
        assert_parity(g_out, oracle_problem(1).evaluate(np.stack(kids)), idx=sel, what=f"colour {c}")
