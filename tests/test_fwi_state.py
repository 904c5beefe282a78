"""The inversion state file: written atomically, read back exactly, with
numpy's loader and no pickled objects."""
import numpy as np
import torch

from paper_2003_06027_amd import fwi


def test_gd_state_round_trip(tmp_path):
    rng = np.random.default_rng(5)
    m = torch.as_tensor(rng.normal(size=(2, 7, 9)).astype(np.float32))
    alpha = torch.tensor([50.0, 31.25], dtype=torch.float64)
    Js = [np.array([1.0, 2.0]), np.array([0.9, 1.7])]
    times = [0.0, 0.25]
    acc = [np.array([True, False])]
    off = [np.array([False, False])]

    class D:
        def state(self):
            return {"off": np.array([True, False]), "consec": np.array([2, 0])}

    p = str(tmp_path / "s.npz")
    fwi.save_gd_state(p, 0, m, alpha, Js, times, acc, off, off, D())
    st = fwi.load_gd_state(p)
    assert int(st["it"]) == 0
    assert np.array_equal(st["models"], m.numpy()) and st["models"].dtype == np.float32
    assert np.array_equal(st["alpha"], alpha.numpy())
    assert np.array_equal(st["J"], np.array(Js)) and np.array_equal(st["accepted"], np.array(acc))
    assert np.array_equal(st["dir_off"], [True, False]) and np.array_equal(st["dir_consec"], [2, 0])
    assert not (tmp_path / "s.npz.tmp.npz").exists()
