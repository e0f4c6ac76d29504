"""The shipped selector model loads without executing anything and has the
network's shape (host only)."""

import os

import numpy as np

import paper_1405_5483_amd as mag_pkg

MODEL = os.path.join(os.path.dirname(mag_pkg.__file__), "selector_model.npz")


def test_model_file_shape_and_values():
    with np.load(MODEL, allow_pickle=False) as z:
        p = z["params"]
        assert p.dtype == np.float32 and p.size == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64
        assert np.isfinite(p).all() and np.abs(p).max() < 1e3
        assert float(z["val_loss"]) < 0.1
