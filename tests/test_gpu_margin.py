"""The re-check margins of the committed weights, re-derived on the GPU.

The classifier runs its layers on MFMA with BF16 or FP16 operands; an
evaluation whose smallest |logit| is below the margin is evaluated again
(BF16 operands: in FP32; FP16 operands: in two-part FP16).  The stated margin of each precision is twice the largest
|z_reduced - z_fp64| over the four logits of 2^20 classifier-training
samples (the samples of Sec. 3.2: half smooth, half step/kink), with the
reduced logits taken at margin 0 from FP32-rounded stencils and the FP64
logits from the oracle on the same stencils.  This test recomputes that
maximum and checks the stored margin against it, and checks on the same
samples that no label decided beyond the margin differs from the FP64 one.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2207_08500_amd import inputs
from tests._helpers import GOLDEN, dev, host, need_gpu, stated_margins, trained_params

pytestmark = pytest.mark.gpu


def test_stated_margins_cover_twice_the_observed_error():
    need_gpu()
    import torch
    from paper_2207_08500_amd import native
    P = trained_params()
    s, _ = inputs.classifier_samples(inputs.BASE_SEED + 100, 1 << 20)
    s32 = s.astype(np.float32).astype(np.float64)
    _, z64 = oracle.mlp_logits(P, s32)
    stated = stated_margins()
    with open(os.path.join(GOLDEN, "neno6_mlp_trained_margins.json")) as f:
        rec = json.load(f)
    for prec, name in ((native.BF16, "bf16"), (native.FP16, "fp16")):
        mlp = native.Mlp(dev(P), recheck_margin=0.0)
        z = torch.zeros((s.shape[0], 4), dtype=torch.float32, device="cuda")
        m = torch.zeros(s.shape[0], dtype=torch.uint8, device="cuda")
        native.neno6_mlp_logits(mlp, prec, dev(s32, torch.float32), z, m)
        torch.cuda.synchronize()
        z = host(z).astype(np.float64)
        dz = np.abs(z - z64)
        flipped = (z > 0) != (z64 > 0)
        depth = np.abs(z)[flipped].max() if flipped.any() else 0.0
        print("%s: max |dz| %.4g (recorded %.4g), margin %.3g, %d flipped logits, deepest "
              "flip |z| %.3g" % (name, dz.max(), rec["observed_max_abs_dz"][name], stated[prec],
                                  int(flipped.sum()), depth))
        assert 2.0 * dz.max() <= stated[prec]
        # the recorded maximum is this one (same samples, same kernels)
        assert abs(dz.max() - rec["observed_max_abs_dz"][name]) <= 1e-3 * rec["observed_max_abs_dz"][name]
        # no label beyond the margin differs from FP64
        assert depth < stated[prec]
