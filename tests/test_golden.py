"""The stored oracle values under tests/golden/ (written by
tests/golden/make_golden.py from the oracle alone) still match the oracle."""

import importlib.util
import json
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load_script():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _walk(a, b, path=""):
    if isinstance(a, dict):
        assert set(a) == set(b), path
        for key in a:
            _walk(a[key], b[key], f"{path}/{key}")
    elif isinstance(a, str):
        assert a == b, path
    else:
        x, y = np.asarray(a, np.float64), np.asarray(b, np.float64)
        assert x.shape == y.shape, path
        assert np.allclose(x, y, rtol=1e-12, atol=1e-300), path


def test_stored_values_match_the_oracle():
    with open(os.path.join(HERE, "oracle_values.json")) as fh:
        stored = json.load(fh)
    _walk(stored, _load_script().compute())
