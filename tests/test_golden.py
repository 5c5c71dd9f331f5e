"""Oracle regression against the stored fixture written by tests/golden/make_golden.py."""

import json
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_tiny_c1_images_regression():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    want = json.load(open(os.path.join(HERE, "tiny_c1_images.json")))
    got = mg.tiny_c1()
    assert got["pixels"] == want["pixels"]
    np.testing.assert_allclose(got["eigenvalues_desc"], want["eigenvalues_desc"], rtol=1e-10, atol=1e-12)
    a = np.array(got["images"])
    b = np.array(want["images"])
    assert np.max(np.abs(a - b)) <= 1e-9 * np.max(np.abs(b))
