"""Shared test helpers: seeded weights and device/host plumbing."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def trained_params() -> np.ndarray:
    """Classifier weights trained by the FP64 oracle (tests/golden/make_weights.py)."""
    return np.load(os.path.join(GOLDEN, "neno6_mlp_trained.npy"), allow_pickle=False)


def stated_margins() -> dict:
    """Re-check margins (logit units) of the committed weights, keyed by the
    library's precision codes (2: BF16, 3: FP16)."""
    import json
    with open(os.path.join(GOLDEN, "neno6_mlp_trained_margins.json")) as f:
        m = json.load(f)["margin"]
    return {2: float(m["bf16"]), 3: float(m["fp16"])}


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def label_flip_rate(ma, mb, nibbles=("lo", "hi")):
    """Fraction of differing candidate labels between two mask-byte arrays."""
    a = np.asarray(ma, np.uint8)
    b = np.asarray(mb, np.uint8)
    x = a ^ b
    bits = np.unpackbits(x.reshape(-1, 1), axis=1)
    n_labels = a.size * 4 * len(nibbles)
    if nibbles == ("lo",):
        bits = bits[:, 4:]
    return bits.sum() / n_labels
