"""The learned preconditioner end to end on the GPU, in the configuration the
benchmark reports (200 training inversions, 20 epochs, 20 evaluation models
x 50 iterations): training data from the plain batched inversion, training with the
library's BF16 kernels, then safeguarded preconditioned descent against
plain descent on unseen models.

The network has no counterpart in the paper, so its effect is "parity
unpinned": what is asserted is what the trained network gains over the
method without it, on data it was not trained on -- the held-out loss
against the true model update falls well below that of the plain direction
(which is what the untrained network returns), and the preconditioned
inversion ends at a lower median misfit than plain descent with the same
step rule and iteration cap, never increasing J."""
import numpy as np
import pytest

from paper_2003_06027_amd import ttm

pytestmark = pytest.mark.gpu


def test_learned_preconditioner_gains_over_plain_descent():
    # A smaller evaluation (8 models x 30 iterations after 10 epochs) left the
    # two medians within 0.2 % of each other, where a change in the rounding
    # of the training data decides the order; the full evaluation separates them.
    cfg = ttm.TTMConfig()
    out = ttm.run(cfg, log=print)
    print({k: v for k, v in out.items()})
    v0, v1 = out["val_loss_untrained_trained"]
    assert v1 < 0.75 * v0
    assert out["train_loss_first_last"][1] < out["train_loss_first_last"][0]
    assert out["cnn_offered_steps"] > 0 and out["cnn_acceptance"] > 0.0
    assert out["cnn_misfit_never_increases"]
    assert out["final_rel_misfit_median_cnn"] < out["final_rel_misfit_median_gd"]
    assert np.isfinite(out["median_seconds_gd"]) and np.isfinite(out["median_seconds_cnn"])
