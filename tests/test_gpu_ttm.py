"""The learned preconditioner end to end on the GPU, in the configuration the
benchmark reports (200 training inversions, 20 epochs, 20 evaluation models
x 150 iterations): training data from the plain batched inversion, training with the
library's BF16 kernels, then safeguarded preconditioned descent against
plain descent on unseen models.

The network has no counterpart in the paper, so its effect is "parity
unpinned": what is asserted is what the trained network gains over the
method without it, on data it was not trained on -- the held-out loss
against the true model update falls well below that of the plain direction
(which is what the untrained network returns); with the misfit target fixed
in advance (J/J0 <= 0.9) the preconditioned inversion reaches it in fewer
median wall-clock seconds than plain descent, on at least as many models,
with the same step rule and iteration cap, never increasing J."""
import numpy as np
import pytest

from paper_2003_06027_amd import ttm

pytestmark = pytest.mark.gpu


def test_learned_preconditioner_gains_over_plain_descent():
    cfg = ttm.TTMConfig()
    assert cfg.tau == 0.9
    out = ttm.run(cfg, log=print)
    print({k: v for k, v in out.items()})
    v0, v1 = out["val_loss_untrained_trained"]
    assert v1 < 0.75 * v0
    assert out["train_loss_first_last"][1] < out["train_loss_first_last"][0]
    assert out["cnn_offered_steps"] > 0 and out["cnn_acceptance"] > 0.0
    assert out["cnn_misfit_never_increases"]
    assert out["final_rel_misfit_median_cnn"] < out["final_rel_misfit_median_gd"]
    # the time-to-misfit claim: the target fixed above, a finite median for
    # the preconditioned descent that beats plain descent's (infinite if fewer
    # than half of the models reach the target), on at least as many models
    assert np.isfinite(out["median_seconds_cnn"])
    assert out["median_seconds_cnn"] < out["median_seconds_gd"]
    assert out["reached_cnn"] >= out["reached_gd"]
    print(f"time to J/J0 <= {cfg.tau}: CNN {out['median_seconds_cnn']:.2f} s ({out['reached_cnn']} models), "
          f"plain {out['median_seconds_gd']:.2f} s ({out['reached_gd']} models); data "
          f"{out['data_seconds']:.1f} s + training {out['train_seconds']:.1f} s")
