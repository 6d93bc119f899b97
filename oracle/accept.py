"""Acceptance of partial solutions in optimal mixing -- plain reference, test
infrastructure only (not part of the library's path).

Sec. 3: a newly sampled partial solution, inserted into its parent, is kept
when the resulting solution dominates the parent or is not dominated within
the current elitist archive.  The three objectives are minimised (Sec. 4.1).

Readings where the paper leaves the details to MO-RV-GOMEA's literature
(listed in the design notes):
  * domination between a child and its parent is constraint domination: a
    feasible solution (no fold in either mesh, valid coordinates) dominates
    an infeasible one; of two infeasible ones the smaller total violation
    (the summed |signed volume| of the violating tets, Sec. 4.1.4 and App. A.4)
    dominates; of two feasible ones Pareto domination decides (no objective
    worse, at least one strictly better);
  * a solution with invalid coordinates, or with an objective or severity
    that is not finite (NaN or an infinity), has infinite violation, so it is
    never accepted;
  * the archive holds feasible solutions; a feasible child is non-dominated
    in it when no member Pareto-dominates it (a member with the same
    objective vector does not); an infeasible child is not accepted through
    the archive;
  * an evaluation whose parent or group index is out of range is never
    accepted;
  * all accepted children of one parent within one batch (elements of one
    colour, whose dependent tets are disjoint) are applied to it;
  * adaptive steering (Sec. 4.3.2) makes a guidance value above the bound
    (1.5 times the archive's best guidance value, chosen by the caller) a
    hard constraint: such a solution is infeasible, and violations compare
    lexicographically as (fold violation, guidance excess), the excess being
    the FP32 difference guidance - bound.  An infinite bound switches it off.
"""
import math

import numpy as np

INVALID = 4
FOLDS = 3


def violation(obj, flags, severity, guidance_max=math.inf):
    """(feasible, violation) of one evaluated solution; the violation is the
    pair (fold violation, guidance excess), compared lexicographically."""
    values = [float(v) for v in obj] + [float(severity)]
    if int(flags) & INVALID or not all(math.isfinite(v) for v in values):
        return False, (math.inf, math.inf)
    folded = bool(int(flags) & FOLDS)
    fold = float(severity) if folded else 0.0
    over = float(obj[2]) > guidance_max
    excess = float(np.float32(np.float32(obj[2]) - np.float32(guidance_max))) if over else 0.0
    return not folded and not over, (fold, excess)


def pareto_dominates(a, b):
    """a is no worse than b in every objective and better in one."""
    return all(x <= y for x, y in zip(a, b)) and any(x < y for x, y in zip(a, b))


def constraint_dominates(a, b, guidance_max=math.inf):
    """a, b: (objectives, flags, severity)."""
    fa, va = violation(*a, guidance_max)
    fb, vb = violation(*b, guidance_max)
    if fa and fb:
        return pareto_dominates(a[0], b[0])
    if fa != fb:
        return fa
    return va < vb


def accept(child, parent, archive, guidance_max=math.inf):
    """child, parent: (objectives, flags, severity); archive: objective vectors."""
    if constraint_dominates(child, parent, guidance_max):
        return True
    feasible, _ = violation(*child, guidance_max)
    return feasible and not any(pareto_dominates(m, child[0]) for m in archive)


def accept_batch(child_obj, child_flags, child_sev, eval_parent, eval_group, n_groups,
                 parent_obj, parent_flags, parent_sev, archive, guidance_max=math.inf):
    """Decision of every evaluation (uint8 0/1)."""
    n_parents = len(parent_flags)
    out = np.zeros(len(child_flags), np.uint8)
    for e in range(len(child_flags)):
        p, g = int(eval_parent[e]), int(eval_group[e])
        if not (0 <= p < n_parents and 0 <= g < n_groups):
            continue
        out[e] = accept((child_obj[e], child_flags[e], child_sev[e]),
                        (parent_obj[p], parent_flags[p], parent_sev[p]), archive, guidance_max)
    return out


def apply(parent_pts, grp_off, grp_pts, eval_parent, eval_group, new_coords, accepted):
    """Parents [n][2][3][n_points] with every accepted evaluation's group points
    set to its new coordinates.  Evaluations with a valid group own
    |group| rows of new_coords ([rows][2][3]) in evaluation order."""
    out = np.array(parent_pts, copy=True)
    n_groups = len(grp_off) - 1
    row = 0
    for e in range(len(eval_parent)):
        g = int(eval_group[e])
        if not 0 <= g < n_groups:
            continue
        idx = grp_pts[grp_off[g]:grp_off[g + 1]]
        if accepted[e]:
            out[int(eval_parent[e])][:, :, idx] = new_coords[row:row + len(idx)].transpose(1, 2, 0)
        row += len(idx)
    return out
