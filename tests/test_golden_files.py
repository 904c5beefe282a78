"""The stored oracle values of the full-length parity tests are current: each
file records the hash of the oracle sources and of the input generator it
was written with (tests/golden/make_long_parity.py), which must match the
tree, and holds the arrays the GPU tests read."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_long_parity as G  # noqa: E402


@pytest.mark.parametrize("name,keys", [
    ("c2", ("pred_sample", "pred_norm2", "obs_norm2", "J", "grad", "shots", "rec_sample")),
    ("c3", ("pred_sample", "pred_norm2", "obs_norm2", "J", "grad_vp", "grad_vs", "grad_rho", "shots", "rec_sample")),
    ("c4", ("pred_sample", "pred_norm2", "obs_norm2", "J", "grad_sub2", "grad_norm2", "grad_probes", "rec_sample")),
])
def test_long_parity_golden_is_current(name, keys):
    path = os.path.join(HERE, "golden", f"long_parity_{name}.npz")
    z = np.load(path)
    assert str(z["oracle_sha256"]) == G.oracle_sha256(), f"stale: rerun tests/golden/make_long_parity.py {name}"
    for k in keys:
        assert k in z.files, k
        assert np.all(np.isfinite(z[k]))
    assert float(z["J"]) > 0 and np.all(z["pred_norm2"] > 0)
