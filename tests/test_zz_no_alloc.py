"""GPU test of the allocation-free DVF entry point (morea_rasterize_dvf_static)
through the C-ABI: its outputs equal those of morea_rasterize_dvf (the same
kernels with a caller workspace) bit for bit, on two calls in a row, the
second on a smaller grid; a grid above the scratch limit is refused with
MOREA_ERANGE before any device work."""
import numpy as np
import pytest

import synth
from conftest import synth_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def outputs(p):
    nx, ny, nz = p.dims
    return dict(fwd=torch.full((nz, ny, nx, 3), np.nan, dtype=torch.float32, device="cuda"),
                inv=torch.full((nz, ny, nx, 3), np.nan, dtype=torch.float32, device="cuda"),
                cover=torch.full((2, nz, ny, nx), -1, dtype=torch.int32, device="cuda"))


def compare(config, seed, folded):
    p = synth_problem(config)
    pop = synth.make_population(p, pop=4, seed=seed, perturb_source=True, fold_fraction=1.0 if folded else 0.0)
    prob = morea.Problem.from_synth(p, max_population=1)
    cand = torch.from_numpy(np.ascontiguousarray(pop[1])).cuda()
    print(f"no-alloc DVF: config {config}, dims {p.dims}, seed {seed}", flush=True)
    want = prob.rasterize_dvf(cand)
    got = prob.rasterize_dvf_static(cand, outputs(p))
    torch.cuda.synchronize()
    for k in ("fwd", "inv", "cover"):
        np.testing.assert_array_equal(got[k].cpu().numpy(), want[k].cpu().numpy(), err_msg=k)
    cover = got["cover"].cpu().numpy()
    assert cover.sum() > 0
    prob.close()
    return cover


def test_static_dvf_equals_workspace_dvf_twice_smaller_second():
    c2 = compare(2, 3, folded=True)            # 128x128x96 (1,572,864 voxels per grid)
    c1 = compare(1, 4, folded=False)           # then 32^3
    assert c2.size > c1.size


def test_static_dvf_refuses_grids_above_the_limit():
    p = synth_problem(4)                        # 192x192x128: 4,718,592 voxels per grid
    prob = morea.Problem.from_synth(p, max_population=1)
    cand = torch.from_numpy(np.ascontiguousarray(synth.make_population(p, pop=1)[0])).cuda()
    out = dict(fwd=torch.empty(1, device="cuda"), inv=torch.empty(1, device="cuda"),
               cover=torch.empty(1, dtype=torch.int32, device="cuda"))
    with pytest.raises(morea.MoreaError) as e:
        prob.rasterize_dvf_static(cand, out)
    assert e.value.status == morea.MOREA_ERANGE
    prob.close()
