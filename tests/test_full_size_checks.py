"""The host-side check used by the full-size GPU test (Eq. 1 recomputed at
sampled vertices from an edge list) against the oracle's fixed point on a
small graph, where Eq. 1 must hold to rounding."""
import importlib.util
import os

import numpy as np

from paper_2407_19562_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _eq1_at():
    spec = importlib.util.spec_from_file_location(
        "full_size_checks", os.path.join(HERE, "test_gpu_full_size.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.eq1_at


def test_eq1_at_fixed_point(oracle_lib):
    eq1_at = _eq1_at()
    n, s, d = inputs.rmat(10, 8 << 10, seed=4)
    R, _, _ = oracle_lib.pagerank(n, s, d)
    vs, r = eq1_at(np.arange(n), n, s, d, R)
    assert np.abs(r - R[vs]).max() < 1e-14
    # a wrong rank is seen
    R2 = R.copy()
    R2[5] *= 1.001
    vs, r = eq1_at(np.array([5, 6, 7]), n, s, d, R2)
    assert np.abs(r - R2[vs]).max() > 1e-8
