"""The oracle against its stored regression values (tests/golden/, written by make_golden.py from
the oracle alone). A change to the oracle's arithmetic that moves these values must name, in its
commit, the passage or reading that justifies it, and regenerate the file."""
import importlib.util
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_oracle_matches_stored_values():
    g = _golden()
    stored = g.read()
    now = g.values()
    for name in ("small", "full"):
        steps = [t for t, _ in stored[name]]
        assert steps == g.STEPS
        ref = np.array([z for _, z in stored[name]])
        got = np.array(now[name])
        # BLAS summation order may differ between hosts: relative 1e-12
        assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(1.0, np.abs(ref))), (name, got - ref)
