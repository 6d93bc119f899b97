import functools
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@functools.lru_cache(maxsize=None)
def synth_problem(config):
    import synth
    return synth.make_problem(config)


@functools.lru_cache(maxsize=None)
def oracle_problem(config):
    import oracle
    return oracle.Problem.from_synth(synth_problem(config))


@pytest.fixture(scope="session")
def c1():
    return synth_problem(1)


@pytest.fixture(scope="session")
def c1_oracle():
    return oracle_problem(1)


def rel_err(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(x - ref) / np.maximum(np.abs(ref), 1e-300)
