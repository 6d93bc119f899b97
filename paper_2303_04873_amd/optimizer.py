"""Generation loop of the optimizer around the evaluator (Sec. 3, Sec. 4.2.1,
Sec. 4.3): a sequence of the library's C-ABI calls on device buffers.  This
module only orders the calls and owns their buffers; every step is a kernel
of libmorea, and the standard normal draws the method consumes come from
torch's generator on the device (inputs of the sampling and repair calls).

One generation:
  1. selection of the population's non-dominated solutions and k clusters
     (morea_select_clusters, under the steering bound);
  2. a snapshot of the population and one normal distribution per
     (cluster, FOS element) (morea_estimate_distributions);
  3. per colour of the linkage model: every (solution, element of the
     colour) child sampled from the solution's cluster with the
     (cluster, element) multiplier (morea_sample_partial), evaluated in one
     batched partial evaluation (morea_eval_partial), accepted against its
     parent and the elitist archive and written back (morea_accept_partial);
     the population then offered to the archive (morea_archive_update) and
     the improvements of the multipliers marked (morea_mark_improvements);
  4. the multipliers adapted (morea_adapt_multipliers);
  5. solutions with a fold repaired (morea_repair_folds, Sec. 4.3.1) and the
     population re-evaluated when any was.
Adaptive steering (Sec. 4.3.2): from generation `steering_at` on, the bound
is fl32(1.5 s_G), s_G the archive's best guidance value after the previous
generation.  The host reads back the population's flags and s_G once per
generation (a few hundred bytes) to decide on the repair and the bound.
"""
from __future__ import annotations

import math

import numpy as np

from . import Archive, build_fos, morea_adapt_multipliers, morea_mark_improvements, select_clusters


class Optimizer:
    def __init__(self, problem, pts, pinned=None, n_clusters=10, selection_fraction=0.35,
                 archive_capacity=2000, steering_at=100, steering_factor=1.5, repair=True, repair_draws=16,
                 seed=0, stream=None):
        import torch
        self.prob = problem
        self.stream = stream
        self.pts = pts                                    # [n][2][3][P] CUDA float32, updated in place
        n = pts.shape[0]
        self.n = n
        self.k = int(n_clusters)
        self.sel_size = int(round(selection_fraction * n))
        self.steering_at = int(steering_at)
        self.steering_factor = np.float32(steering_factor)
        self.repair = bool(repair)
        self.repair_draws = int(repair_draws)
        self.pinned = pinned
        elements, colors, n_colors = build_fos(problem.n_points, problem.tets_host)
        self.elements, self.colors = elements, colors
        off = np.arange(0, 2 * len(elements) + 1, 2, dtype=np.int32)
        problem.set_groups(off, elements.reshape(-1).astype(np.int32))
        self.n_groups = len(elements)
        per_colour = [np.flatnonzero(colors == c).astype(np.int32) for c in range(n_colors)]
        problem.reserve_partial(n * max(len(g) for g in per_colour))
        self.gen = torch.Generator(device="cuda")
        self.gen.manual_seed(int(seed))
        self.batches = []
        for g in per_colour:
            ep = np.repeat(np.arange(n, dtype=np.int32), len(g))
            eg = np.tile(g, n)
            dep = torch.from_numpy(ep).cuda()
            self.batches.append(dict(
                ep=ep, eg=eg, dep=dep, dep_long=dep.long(), deg=torch.from_numpy(eg).cuda(),
                ec=torch.empty(len(ep), dtype=torch.int32, device="cuda"),
                z=torch.empty((2 * len(ep), 2, 3), dtype=torch.float32, device="cuda"),
                new=torch.empty((2 * len(ep), 2, 3), dtype=torch.float32, device="cuda"),
                out=problem.outputs(len(ep)), acc=torch.empty(len(ep), dtype=torch.uint8, device="cuda")))
        self.snap = torch.empty_like(pts)
        self.work = problem.mixing_workspace(self.k)
        self.cache = problem.new_cache(n)
        self.out = problem.eval_full(pts, cache=self.cache, stream=stream)
        self.archive = Archive(archive_capacity, n_points=problem.n_points, stream=stream)
        self.inserted = torch.empty(n, dtype=torch.uint8, device="cuda")
        self.slot_of = torch.empty(n, dtype=torch.int32, device="cuda")
        self.mult = torch.ones((self.k, self.n_groups), dtype=torch.float32, device="cuda")
        self.nis = torch.zeros((self.k, self.n_groups), dtype=torch.int32, device="cuda")
        self.improved = torch.zeros((self.k, self.n_groups), dtype=torch.uint8, device="cuda")
        self.draws = torch.empty((n, self.repair_draws, 64, 3), dtype=torch.float32, device="cuda")
        self.generation = 0
        self.repaired = 0
        self.bound = math.inf
        self.s_g = math.inf
        self._repair_and_offer(initial=True)

    def _sync_state(self):
        """One small read-back: the population's flags and the archive's best
        guidance value."""
        import torch
        torch.cuda.synchronize()
        flags = self.out["flags"].cpu().numpy()
        self.s_g = float(self.archive.best.cpu().numpy()[0])
        return flags

    def _repair_and_offer(self, initial=False):
        """Repair the solutions with a fold and re-evaluate the population when
        any was repaired; offer the population to the archive when it changed
        (and at the start)."""
        flags = self._sync_state()
        folded = ((flags & 3) != 0) & ((flags & 4) == 0)
        self.folded_before_repair = int(folded.sum())
        changed = False
        if self.repair and folded.any():
            self.draws.normal_(generator=self.gen)
            self.info = self.prob.repair_folds(self.pts, self.draws, pinned=self.pinned, stream=self.stream)
            self.prob.eval_full(self.pts, cache=self.cache, out=self.out, stream=self.stream)
            self.repaired += int(folded.sum())
            changed = True
        if changed or initial:
            gmax = None if math.isinf(self.bound) else self.bound
            self.archive.update(self.out, pts=self.pts, guidance_max=gmax, inserted=self.inserted,
                                slot_of=self.slot_of, stream=self.stream)
            self._sync_state()

    def steering_bound(self):
        if self.generation < self.steering_at or not math.isfinite(self.s_g):
            return math.inf
        return float(self.steering_factor * np.float32(self.s_g))

    def step(self, record=None):
        """One generation.  With `record` (a dict), host copies of what the
        generation drew and decided are stored in it for inspection: the
        bound, the selection, per colour the draws, samples, child outputs,
        decisions, clusters, the parents' outputs and the archive after the
        colour's update, then the multipliers and the repair's draws."""
        self.bound = self.steering_bound()
        gmax = None if math.isinf(self.bound) else self.bound
        sc = select_clusters(self.out, self.sel_size, self.k, guidance_max=gmax, stream=self.stream)
        self.snap.copy_(self.pts)
        self.prob.estimate_distributions(self.snap, sc["clu_off"], sc["clu_members"], self.work, pinned=self.pinned,
                                         stream=self.stream)
        self.selection = sc
        if record is not None:
            record["bound"] = self.bound
            record["selection"] = {k: v.cpu().numpy() for k, v in sc.items()}
            record["colours"] = []
        self.kept = 0
        for b in self.batches:
            b["z"].normal_(generator=self.gen)
            b["ec"].copy_(sc["cluster_of"][b["dep_long"]])
            self.prob.sample_partial(self.pts, self.work, self.k, b["dep"], b["deg"], b["ec"], b["z"],
                                     pinned=self.pinned, mult=self.mult, out=b["new"], stream=self.stream)
            self.prob.eval_partial(self.pts, self.cache, b["dep"], b["deg"], b["new"], out=b["out"],
                                   stream=self.stream)
            self.prob.accept_partial(self.pts, self.cache, b["dep"], b["deg"], b["new"], b["out"], self.out,
                                     archive=self.archive.obj, guidance_max=gmax, accepted=b["acc"],
                                     stream=self.stream)
            self.archive.update(self.out, pts=self.pts, guidance_max=gmax, inserted=self.inserted,
                                slot_of=self.slot_of, stream=self.stream)
            morea_mark_improvements(b["dep"], b["deg"], b["ec"], b["acc"], self.inserted, self.improved,
                                    stream=self.stream)
            if record is not None:
                host = lambda d: {k: v.cpu().numpy() for k, v in d.items()}   # noqa: E731
                record["colours"].append(dict(
                    z=b["z"].cpu().numpy(), new=b["new"].cpu().numpy(), acc=b["acc"].cpu().numpy(),
                    ec=b["ec"].cpu().numpy(), out=host(b["out"]), parents=host(self.out),
                    pts=self.pts.cpu().numpy(), inserted=self.inserted.cpu().numpy(),
                    slot_of=self.slot_of.cpu().numpy(), stamp=self.archive.stamp.cpu().numpy(),
                    arc_obj=self.archive.obj.cpu().numpy(), state=self.archive.state.cpu().numpy()))
        morea_adapt_multipliers(self.improved, self.mult, self.nis, stream=self.stream)
        self.generation += 1
        self._repair_and_offer()
        if record is not None:
            record["mult"] = self.mult.cpu().numpy()
            record["nis"] = self.nis.cpu().numpy()
            record["repaired"] = self.folded_before_repair if self.repair else 0
            record["draws"] = self.draws.cpu().numpy() if self.repair and self.folded_before_repair else None
            record["pts"] = self.pts.cpu().numpy()
            record["stamp"] = self.archive.stamp.cpu().numpy()
            record["s_g"] = self.s_g
