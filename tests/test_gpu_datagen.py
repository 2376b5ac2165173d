"""The training-data generator (Alg. 1, appendix function families) on the
GPU: evolution and TENO6-opt labels go through the library; every
TENO-labelled sample must carry exactly the oracle's TENO6-opt labels of its
stencil, and training on the generated set lowers the loss."""
import numpy as np
import pytest

import oracle
from tests._helpers import dev, host, need_gpu

pytestmark = pytest.mark.gpu


def test_generated_labels_and_training():
    need_gpu()
    import torch
    from paper_2207_08500_amd import datagen, inputs, native
    s, y, kind = datagen.generate(6000, seed=12)
    assert s.shape == (6000, 6) and y.shape == (6000,) and np.all(y <= 15)
    assert np.all(np.isfinite(s))
    assert set(np.unique(kind).tolist()) == {0, 1, 2}
    teno = kind > 0
    _, _, _, m = oracle.teno(s[teno])
    assert np.array_equal(y[teno], (~m) & 15)
    frac = (y != 0).mean()
    print("generated: %d samples, kinds %s, flagged fraction %.3f"
          % (s.shape[0], np.bincount(kind).tolist(), frac))
    assert 0.02 < frac < 0.9
    # a short FP32 training run on the generated data lowers the BCE loss
    P = dev(inputs.mlp_init(7))
    mm = torch.zeros(3228, dtype=torch.float64, device="cuda")
    vv = torch.zeros(3228, dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    sg, yg = dev(s, torch.float32), dev(y)
    hist = []
    step = 0
    for ep in range(6):
        perm = dev(np.random.default_rng(ep).permutation(6000))
        step = native.neno6_classifier_train(P, mm, vv, step, sg, yg, perm, 256, 3e-3,
                                             precision=native.FP32, loss_out=loss)
        torch.cuda.synchronize()
        hist.append(float(host(loss)[0]))
    print("loss per epoch", hist)
    assert hist[-1] < 0.8 * hist[0]
