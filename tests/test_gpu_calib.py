"""VALU issue-rate calibration (mg_valu_rate) on the GPU: every instruction
kind runs and reports a rate no SIMD can exceed (one wave64 instruction per
SIMD and cycle at the 2.4 GHz peak engine clock, 256 CUs of 4 SIMDs: 157.3e12
lane-ops/s), with 5 % allowance for the event timer."""
import pytest

pytestmark = pytest.mark.gpu

CEILING = 256 * 4 * 64 * 2.4e9 * 1.05


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_02175_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("op", [0, 1, 2, 3, 4, 5])
def test_valu_rate_runs_below_the_issue_ceiling(B, op):
    print(f"valu rate: op={op}", flush=True)
    rate, ms = B.mg_valu_rate(op, 8, 4096)
    assert ms > 0.0
    assert 0.0 < rate <= CEILING, rate
