"""The device generator of seeded training samples against its host twin
(the input module's Philox4x32-10 recipe): labels bit for bit (they are
decided by FP64 comparisons of positions both sides form with the same
separately rounded operations), stencil values bit for bit where no
transcendental function is involved (polynomials, steps) and within one
FP32 rounding otherwise (the device's exp and sin may differ from the
host's in the last FP64 bit)."""
import numpy as np
import pytest

from paper_2207_08500_amd import inputs
from tests._helpers import host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("first,n", [(0, 1), (0, 257), (12345, 100003), ((1 << 24) - 100, 200),
                                     ((1 << 33) + 7, 1000)])
def test_device_samples_equal_host_twin(first, n):
    need_gpu()
    import torch
    from paper_2207_08500_amd import native
    native.load()
    seed = inputs.BASE_SEED + 5
    s_h, y_h, s64 = inputs.classifier_samples_philox(seed, first, n)
    s_d, y_d = native.neno6_classifier_samples(seed, first, n)
    torch.cuda.synchronize()
    s_d, y_d = host(s_d), host(y_d)
    assert np.array_equal(y_d, y_h)
    exact = np.array_equal(s_d.view(np.uint32), s_h.view(np.uint32))
    ulp = np.spacing(np.abs(s_h).astype(np.float32))
    assert np.all(np.abs(s_d - s_h) <= ulp), np.abs(s_d - s_h).max()
    print("first %d n %d: labels equal, values %s" % (first, n, "bitwise" if exact else "within 1 ulp"))


def test_device_samples_refuse_bad_sizes():
    need_gpu()
    import torch
    from paper_2207_08500_amd import native
    native.load()
    with pytest.raises(native.Neno6Error):
        native.neno6_classifier_samples(1, -1, 4)
    s, y = native.neno6_classifier_samples(1, 0, 0)
    assert s.numel() == 0 and y.numel() == 0
