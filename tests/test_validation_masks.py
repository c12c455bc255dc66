"""The validation harness's masks: exact removal counts, determinism per (seed, p, m), and distinct masks."""
import numpy as np

from paper_2212_01317_amd import synth


def test_masks_exact_and_deterministic():
    import importlib
    v = importlib.import_module("paper_2212_01317_amd.validation")
    a = v.masks_for(31, 45, 0.3, 3, seed=7)
    b = v.masks_for(31, 45, 0.3, 3, seed=7)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert all(int((m == 0).sum()) == round(0.3 * 31 * 45) for m in a)
    assert not np.array_equal(a[0], a[1])


def test_skewed_field_skewness():
    f = synth.skewed_field(256, 11).astype(np.float64)
    g = (f - f.mean()) / f.std()
    skew = float(np.mean(g ** 3))
    assert np.all(f > 0) and 2.0 < skew < 5.5
