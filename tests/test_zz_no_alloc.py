"""The allocation-free misfit (misfit_noalloc, partial sums in the library's
static device array) against the model's misfit (partial sums in the model's
workspace) through the C ABI: J and the residual bitwise equal, on two calls
in a row, the second with a smaller input, then on degenerate sizes; and the
size limit refused before any launch."""
import numpy as np
import pytest
import torch

from gpu_common import S, synth, dev, gpu_desc

pytestmark = pytest.mark.gpu


def _noalloc(pred, obs):
    J = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    r = torch.full_like(pred, -7.0)
    rc = S.lib().misfit_noalloc(S._ptr(pred), S._ptr(obs), pred.numel(), S._ptr(J), S._ptr(r), S._stream())
    assert rc == S.SG_OK, S.lib().last_error().decode()
    return J, r


def test_noalloc_misfit_equals_model_misfit_bitwise():
    m = S.Model(gpu_desc(synth.C1, 3000.0), dev(synth.layered_c1()), 1, 101)
    rng = np.random.default_rng(11)
    for n in (3_000_001, 100_003, 4096, 5, 1):       # the second call is smaller than the first
        a = rng.standard_normal(n).astype(np.float32)
        b = rng.standard_normal(n).astype(np.float32)
        pa, pb = dev(a), dev(b)
        J_ref, r_ref = m.misfit(pa, pb)
        J_na, r_na = _noalloc(pa, pb)
        torch.cuda.synchronize()
        assert J_na.item() == J_ref.item(), (n, J_na.item(), J_ref.item())
        assert torch.equal(r_na, r_ref)
        r32 = (a - b).astype(np.float64)
        assert J_na.item() == pytest.approx(0.5 * np.dot(r32, r32), rel=1e-12)
    # n = 0: J = 0 with NULL inputs
    J = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    assert S.lib().misfit_noalloc(None, None, 0, S._ptr(J), None, S._stream()) == S.SG_OK
    torch.cuda.synchronize()
    assert J.item() == 0.0
    # beyond the stated maximum (2^40 elements) and negative sizes: refused on the host
    x = torch.zeros(4, device="cuda")
    assert S.lib().misfit_noalloc(S._ptr(x), S._ptr(x), (1 << 40) + 1, S._ptr(J), None, S._stream()) == S.SG_EINVAL
    assert b"2^40" in S.lib().last_error()
    assert S.lib().misfit_noalloc(S._ptr(x), S._ptr(x), -1, S._ptr(J), None, S._stream()) == S.SG_EINVAL
    m.close()
