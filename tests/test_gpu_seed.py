"""The device generator of the seeded initial density (lbm_seeded_density,
SplitMix64 per node) against the host generator of the same published
definition (synth.noisy_density): bit-identical fields."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def glbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_0905_amd import lbm
    lbm.load_library()
    return lbm


@pytest.mark.parametrize("shape,seed,rho,amp", [((32, 32, 32), 1234, 1.17881, 0.01),
                                                ((7, 5, 3), 0, 2.49, 0.3),
                                                ((130, 1, 9), 2 ** 63 + 12345, 1.0, 0.999)])
def test_device_field_equals_host_field(glbm, shape, seed, rho, amp):
    nx, ny, nz = shape
    want = synth.noisy_density(nx, ny, nz, rho, amp, seed)
    got = glbm.lbm_seeded_density(nx, ny, nz, seed, rho, amp)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)


def test_invalid_arguments(glbm):
    with pytest.raises(glbm.LbmError):
        glbm.lbm_seeded_density(4, 4, 4, 1, 1.0, 1.5)
    with pytest.raises(glbm.LbmError):
        glbm.lbm_seeded_density(4, 4, 4, 1, -1.0, 0.1)
