"""Each plausible mistake planted in the oracle (on the CPU, in a copy of its
C source) must make at least one pin fail: the pins constrain every part of
the definition, not only the code paths they happen to call."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "morea_oracle.c")

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
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                           str(mutant), "-lm"])
    env = dict(os.environ, MOREA_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught: {name}\n{r.stdout[-2000:]}"
