"""Each plausible mistake planted in the oracle (on the CPU, in a copy of its
C source, or of its Python references for fold repair and the linkage model)
must make at least one pin fail: the pins constrain every part of the
definition, not only the code paths they happen to call."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "morea_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")
SOBOL = os.path.join(ROOT, "tests", "test_oracle_sobol.py")
DVF = os.path.join(ROOT, "tests", "test_oracle_dvf.py")
POINTS = os.path.join(ROOT, "tests", "test_oracle_point_guidance.py")

MUTATIONS = [
    ("directions swapped in the target->source pass",
     "eval_direction(P, T, S, ref[t], 1, w_t, &recs[2 * it + 1]);",
     "eval_direction(P, S, T, ref[t], 1, w_t, &recs[2 * it + 1]);"),
    ("tie rule with the opposite sign",
     "int pos = grad[0] > 0 || (grad[0] == 0 && (grad[1] > 0 || (grad[1] == 0 && grad[2] > 0)));",
     "int pos = grad[0] < 0 || (grad[0] == 0 && (grad[1] < 0 || (grad[1] == 0 && grad[2] < 0)));"),
    ("spokes dropped from the magnitude",
     "    double d = edge_len(s4, cs, 4.0 * FIX_ONE) - edge_len(t4, ct, 4.0 * FIX_ONE);\n    acc += d * d;",
     "    double d = edge_len(s4, cs, 4.0 * FIX_ONE) - edge_len(t4, ct, 4.0 * FIX_ONE);\n    acc += 0.0 * d;"),
    ("foreground/background mismatch costs 0.5",
     "          h = 1.0;", "          h = 0.5;"),
    ("guidance without the (r - d) / r weight",
     "rec->g += set_w[s] * ((r - d) / r) * (d - d2) * (d - d2);",
     "rec->g += set_w[s] * (d - d2) * (d - d2);"),
    ("guidance without the set weights",
     "rec->g += set_w[s] * ((r - d) / r) * (d - d2) * (d - d2);",
     "rec->g += ((r - d) / r) * (d - d2) * (d - d2);"),
    ("intensity normalised by |P_s| only",
     "obj[3 * c + 0] = H / N;", "obj[3 * c + 0] = H / (double)Ns;"),
    ("trilinear weights reversed",
     "double w = (dx ? f[0] : 1.0 - f[0]) *", "double w = (dx ? 1.0 - f[0] : f[0]) *"),
    ("interpolated foreground from all 8 corners (no exact support)",
     "for (int dz = 0; dz <= !exact[2]; dz++)", "for (int dz = 0; dz <= 1; dz++)"),
    ("zero volume not a fold",
     "rec->viol = (sgn128(D) == 0) || (sgn128(D) != ref_sign);",
     "rec->viol = (sgn128(D) != 0) && (sgn128(D) != ref_sign);"),
    ("magnitude normalised by 6 |Delta|",
     "obj[3 * c + 1] = M / (10.0 * (double)NT);", "obj[3 * c + 1] = M / (6.0 * (double)NT);"),
    ("zero padding replaced by edge clamping for intensities",
     "              : fetch_zero(img, nx, ny, nz, k[0] + dx, k[1] + dy, k[2] + dz);",
     "              : fetch_clamp(img, nx, ny, nz, k[0] + dx, k[1] + dy, k[2] + dz);"),
    ("guidance band with <= instead of <",
     "if (!(d < r)) continue;", "if (!(d <= r + 0.5)) continue;"),
    # the Sobol-sampled estimator, against its own pins
    ("Sobol: barycentric coordinates not normalised by the sum",
     "const float l1 = e[1] / sum, l2 = e[2] / sum, l3 = e[3] / sum;",
     "const float l1 = e[1] / (sum + e[0]), l2 = e[2] / (sum + e[0]), l3 = e[3] / (sum + e[0]);", SOBOL),
    ("Sobol: mapped point built from the sampled tet's edges",
     "q[a] = fmaf(l3, edge_oth[2][a], fmaf(l2, edge_oth[1][a], fmaf(l1, edge_oth[0][a], base_oth[a])));",
     "q[a] = fmaf(l3, edge_own[2][a], fmaf(l2, edge_own[1][a], fmaf(l1, edge_own[0][a], base_oth[a])));", SOBOL),
    ("Sobol: wrong ln 2 in -log",
     "return -fmaf((float)k, 0x1.62e430p-1f, ln_m);", "return -fmaf((float)k, 0x1.6p-1f, ln_m);", SOBOL),
    ("Sobol: series of atanh cut after s^3",
     "poly = fmaf(t, poly, 0x1.99999ap-3f);", "poly = 0x1.99999ap-3f;", SOBOL),
    ("Sobol: guidance without the (r - d) / r weight",
     "rec->g += set_w[s] * (radius - d_own) / radius * diff * diff;",
     "rec->g += set_w[s] * diff * diff;", SOBOL),
    ("Sobol: sample count truncated instead of rounded",
     "const double x = floor((double)absD * scale + 0.5);", "const double x = floor((double)absD * scale);",
     SOBOL),
    ("Sobol: no digital shift",
     "const uint32_t u = sobol_coord(j, n) ^ shift[j];", "const uint32_t u = sobol_coord(j, n);", SOBOL),
    ("Sobol: wrong primitive polynomial for the fourth dimension",
     "const uint32_t inner[4] = {0, 0, 1, 1};", "const uint32_t inner[4] = {0, 0, 1, 0};", SOBOL),
    ("Sobol: foreground/background mismatch costs 0.5",
     "(fa == fb ? 0.0 : 1.0)", "(fa == fb ? 0.0 : 0.5)", SOBOL),
    ("Sobol: own image read at the mapped point",
     "const double a = fa ? trilinear(img_own, P->nx, P->ny, P->nz, kp, fp, 0) : 0.0;",
     "const double a = fa ? trilinear(img_own, P->nx, P->ny, P->nz, kq, fq, 0) : 0.0;", SOBOL),
    # deformation vector fields and the point-based guidance error
    ("DVF: displacement p - q instead of q - p",
     "out[3 * v + a] = (double)(kq[a] - pv[a]) + fq[a];", "out[3 * v + a] = (double)(pv[a] - kq[a]) - fq[a];", DVF),
    ("DVF: the last covering tet owns a centre",
     "if (owner[v] >= 0) continue;", "if (owner[v] > t) continue;", DVF),
    ("point guidance: distance instead of squared distance",
     "        total += best;", "        total += sqrt(best);", POINTS),
    ("point guidance: every tet's bounding box taken as containing the point",
     "if (!inside_tie(S, D, cp, lam)) continue;", "(void)inside_tie(S, D, cp, lam);", POINTS),
]

# mistakes planted in copies of the Python references, each run against its pins
REPAIR = os.path.join(ROOT, "tests", "test_oracle_repair.py")
FOS = os.path.join(ROOT, "tests", "test_oracle_fos.py")
ACCEPT = os.path.join(ROOT, "tests", "test_oracle_accept.py")
MIXING = os.path.join(ROOT, "tests", "test_oracle_mixing.py")
SELECTION = os.path.join(ROOT, "tests", "test_oracle_selection.py")
QUANT = os.path.join(ROOT, "tests", "test_oracle_quantize.py")
PY_MUTATIONS = [
    ("quantize: BF16 truncated", "__init__.py", "rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16",
     "rounded = u >> 16", QUANT, []),
    ("quantize: BF16 ties away from zero", "__init__.py", "rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16",
     "rounded = (u + 0x8000) >> 16", QUANT, []),
    ("repair: step twice the rounded-down distance", "repair.py",
     "while j < SIGMA_MAX_LOG2 and (4 ** (j + 1)) * n * n <= d2:",
     "while j < SIGMA_MAX_LOG2 and (4 ** j) * n * n <= d2:", REPAIR, []),
    ("repair: a tie aborts the candidate", "repair.py",
     "elif best is not None and best[0] == c0:", "elif False:", REPAIR, []),
    ("repair: pinned axes move", "repair.py",
     "if not (fixed is not None and (int(fixed[v]) >> a) & 1):", "if True:", REPAIR, []),
    ("repair: constraint without the folded volume", "repair.py", "sev += abs(D)", "sev += 0", REPAIR, []),
    ("repair: points visited in descending order", "repair.py",
     "todo += [(m, v) for v in sorted(pts)]", "todo += [(m, v) for v in sorted(pts, reverse=True)]", REPAIR, []),
    ("fos: DSATUR ties to the smaller degree", "fos.py",
     "return (sat, len(adj[v]), -v)", "return (sat, -len(adj[v]), -v)", FOS, ["-k", "not 2"]),
    ("fos: interaction only between elements sharing a point", "fos.py",
     "deps = [holding.get(a, set()) | holding.get(b, set()) for a, b in elements]",
     "deps = [{-1 - a, -1 - b} for a, b in elements]", FOS, ["-k", "not 2"]),
    ("fos: set cover prefers the last of equally good edges", "fos.py",
     "if g > gain:", "if g >= gain and g > 0:", FOS, ["-k", "not 2"]),
    ("accept: weak Pareto domination", "accept.py",
     "and any(x < y for x, y in zip(a, b))", "", ACCEPT, []),
    ("accept: infeasible preferred over feasible", "accept.py", "        return fa\n", "        return fb\n",
     ACCEPT, []),
    ("accept: equal violations dominate", "accept.py", "return va < vb", "return va <= vb", ACCEPT, []),
    ("accept: archive test reversed", "accept.py",
     "pareto_dominates(m, child[0]) for m in archive", "pareto_dominates(child[0], m) for m in archive", ACCEPT, []),
    ("accept: infeasible children through the archive", "accept.py",
     "return feasible and not any(", "return not any(", ACCEPT, []),
    ("accept: NaN objectives count as feasible", "accept.py",
     "if int(flags) & INVALID or not all(math.isfinite(v) for v in values):", "if int(flags) & INVALID:", ACCEPT, []),
    ("accept: infinite objectives count as feasible", "accept.py",
     "if int(flags) & INVALID or not all(math.isfinite(v) for v in values):",
     "if int(flags) & INVALID or any(math.isnan(v) for v in values):", ACCEPT, []),
    ("selection: infinite objectives selected", "selection.py",
     "and all(math.isfinite(float(v)) for v in list(obj) + [severity])",
     "and not any(math.isnan(float(v)) for v in list(obj) + [severity])", SELECTION, []),
    ("accept: rows owned by accepted evaluations only", "accept.py",
     "            out[int(eval_parent[e])][:, :, idx] = new_coords[row:row + len(idx)].transpose(1, 2, 0)\n"
     "        row += len(idx)",
     "            out[int(eval_parent[e])][:, :, idx] = new_coords[row:row + len(idx)].transpose(1, 2, 0)\n"
     "            row += len(idx)", ACCEPT, []),
    ("steering: excess outranks folds", "accept.py", "return not folded and not over, (fold, excess)",
     "return not folded and not over, (excess, fold)", ACCEPT, []),
    ("steering: bound ignored for feasibility", "accept.py", "return not folded and not over, (fold, excess)",
     "return not folded, (fold, excess)", ACCEPT, []),
    ("steering: bound itself outside", "accept.py", "over = float(obj[2]) > guidance_max",
     "over = float(obj[2]) >= guidance_max", ACCEPT, []),
    ("selection: last front cut from the highest index", "selection.py",
     "chosen += [i for i in range(len(rank)) if rank[i] == r][:size - len(chosen)]",
     "chosen += [i for i in range(len(rank)) if rank[i] == r][::-1][:size - len(chosen)]", SELECTION, []),
    ("selection: objectives not normalised", "selection.py",
     "return [((float(v[o]) - lo[o]) / (hi[o] - lo[o])) if hi[o] > lo[o] else 0.0 for o in range(3)]",
     "return [(float(v[o]) - lo[o]) for o in range(3)]", SELECTION, []),
    ("selection: first leader of largest first objective", "selection.py",
     "first = min(sel, key=lambda i: (pts[i][0], i))", "first = max(sel, key=lambda i: (pts[i][0], -i))",
     SELECTION, []),
    ("selection: distance to the last leader only", "selection.py", "            if d < nearest[i]:",
     "            if True:", SELECTION, []),
    ("selection: clusters of |S| / k", "selection.py", "m = min(len(sel), -(-2 * len(sel) // k))",
     "m = min(len(sel), -(-len(sel) // k))", SELECTION, []),
    ("selection: ties to the higher cluster", "selection.py",
     "key=lambda j: (dist(pts[i], pts[leaders[j]]), j)))", "key=lambda j: (dist(pts[i], pts[leaders[j]]), -j)))",
     SELECTION, []),
    ("mixing: unbiased covariance", "mixing.py", "cov[u][v] = cov[v][u] = s / m", "cov[u][v] = cov[v][u] = s / (m - 1)",
     MIXING, []),
    ("mixing: mean over m + 1", "mixing.py", "mean.append(s / m)", "mean.append(s / (m + 1))", MIXING, []),
    ("mixing: factor row uses its own entries", "mixing.py", "s = s - L[i][k] * L[j][k]", "s = s - L[i][k] * L[i][k]",
     MIXING, []),
    ("mixing: multiplier scales the deviation", "mixing.py", "scale = math.sqrt(float(np.float32(mult)))",
     "scale = float(np.float32(mult))", MIXING, []),
    ("mixing: diagonal term left out of the sample", "mixing.py", "for k in range(u + 1):", "for k in range(u):",
     MIXING, []),
    ("mixing: fallback uses variances", "mixing.py", "L[i][i] = math.sqrt(cov[i][i])", "L[i][i] = cov[i][i]",
     MIXING, []),
    ("mixing: pinned axes sampled", "mixing.py", "if pinned is None or not (int(pinned[pt]) >> a) & 1:", "if True:",
     MIXING, []),
]


@pytest.mark.parametrize("name,old,new,pins", [m if len(m) == 4 else m + (PINS,) for m in MUTATIONS],
                         ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, pins, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", str(lib), str(mutant), "-lm"])
    env = dict(os.environ, MOREA_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught: {name}\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name,fname,old,new,pins,args", PY_MUTATIONS, ids=[m[0] for m in PY_MUTATIONS])
def test_planted_python_mistake_is_caught(name, fname, old, new, pins, args, tmp_path):
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg, ignore=shutil.ignore_patterns("__pycache__"))
    src = (pkg / fname).read_text()
    assert src.count(old) == 1, name
    (pkg / fname).write_text(src.replace(old, new))
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([str(tmp_path), ROOT]), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", pins] + args,
                       cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught: {name}\n{r.stdout[-2000:]}"
