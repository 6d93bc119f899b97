"""Helpers shared by the GPU parity tests: run the HIP path through the C-ABI
binding and compare with the oracle to the parity bar.

The bar: sample counts and flags bit-exact; every objective and the severity
within 1e-5 relative of the FP64 oracle (values whose oracle value is 0 must
be within 1e-6 absolute)."""
import numpy as np

REL_TOL = 1e-5
ABS_TOL_ZERO = 1e-6


def to_host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def assert_parity(gpu, ora, idx=None, rel_tol=REL_TOL, what=""):
    """gpu: host dict from the binding; ora: oracle dict; idx: oracle rows
    correspond to gpu rows idx (default all)."""
    idx = np.arange(len(ora["flags"])) if idx is None else np.asarray(idx)
    g_obj = gpu["obj"][idx].astype(np.float64)
    o_obj = ora["obj"]
    np.testing.assert_array_equal(gpu["flags"][idx], ora["flags"], err_msg=f"flags {what}")
    np.testing.assert_array_equal(gpu["counts"][idx].astype(np.int64), ora["counts"],
                                  err_msg=f"counts {what}")
    inv = (ora["flags"] & 4) != 0
    assert np.all(np.isnan(g_obj[inv])), what
    ok = ~inv
    for name, g, o in [("obj", g_obj[ok], o_obj[ok]),
                       ("severity", gpu["severity"][idx][ok].astype(np.float64), ora["severity"][ok])]:
        zero = o == 0
        assert np.all(np.abs(g[zero]) <= ABS_TOL_ZERO), (name, what, g[zero])
        rel = np.abs(g[~zero] - o[~zero]) / np.abs(o[~zero])
        worst = rel.max() if rel.size else 0.0
        assert worst <= rel_tol, f"{name} {what}: worst rel err {worst:.3e}"
    return worst_rel(gpu, ora, idx)


def worst_rel(gpu, ora, idx):
    g = gpu["obj"][idx].astype(np.float64)
    o = ora["obj"]
    ok = ((ora["flags"] & 4) == 0)[:, None] & (o != 0)
    rel = np.where(ok, np.abs(g - o) / np.where(o == 0, 1, np.abs(o)), 0.0)
    return rel.max(axis=0)
