"""The allocation-free right-hand side (neno6_rhs_noalloc) against neno6_rhs.

Both run the same fused kernel; the no-alloc entry point keeps the face ->
line map in a static device array instead of the caller's workspace.  Its
outputs (right-hand side, kept masks, status words) must equal neno6_rhs's
bit for bit, on two calls in a row where the second batch is smaller than
the first (the array then still holds the first batch's map past the second
one's end), after which a call flagged "map kept" must still rebuild the map.
A batch beyond the array's capacity is refused before anything is enqueued,
and an unsupported equation or precision is refused.
"""
import numpy as np
import pytest

from paper_2207_08500_amd import inputs
from tests._helpers import need_gpu, trained_params

pytestmark = pytest.mark.gpu


def _batch(seed, sizes):
    q, off, dx = inputs.riemann1d_batch(seed, np.asarray(sizes, np.int64), perturb=True)
    return q, off, dx


def _compare(native, torch, P, prec, margin, q, off, dx, keep_map=False):
    d = torch.device("cuda:0")
    mlp = native.Mlp(torch.as_tensor(P, device=d), recheck_margin=margin)
    prob = native.Problem(native.EULER1D, prec, native.SEL_MLP, native.TRANSMISSIVE, off, dx,
                          device=d)
    q32 = torch.as_tensor(q, dtype=torch.float32, device=d).contiguous()
    nprob = off.size - 1
    # reference: neno6_rhs with its own workspace
    ws = prob.workspace(d)
    r_ref = torch.zeros_like(q32)
    m_ref = torch.zeros(prob.mask_count(), dtype=torch.uint8, device=d)
    s_ref = torch.zeros(nprob, dtype=torch.int32, device=d)
    native.neno6_rhs(prob, mlp, q32, r_ref, ws, masks_out=m_ref, status=s_ref)
    # the no-alloc entry point (outputs pre-filled with garbage)
    r = torch.full_like(q32, float("nan"))
    m = torch.full((prob.mask_count(),), 0xA5, dtype=torch.uint8, device=d)
    s = torch.zeros(nprob, dtype=torch.int32, device=d)
    if keep_map:
        prob.flags = native.KEEP_MAP  # ignored by the no-alloc entry point
    native.neno6_rhs_noalloc(prob, mlp, q32, r, masks_out=m, status=s)
    torch.cuda.synchronize()
    assert torch.equal(r.view(torch.int32), r_ref.view(torch.int32))
    assert torch.equal(m, m_ref)
    assert torch.equal(s, s_ref)
    # and without masks (the path the step takes)
    r2 = torch.full_like(q32, float("nan"))
    native.neno6_rhs_noalloc(prob, mlp, q32, r2)
    r2_ref = torch.zeros_like(q32)
    prob.flags = 0
    native.neno6_rhs(prob, mlp, q32, r2_ref, ws)
    torch.cuda.synchronize()
    assert torch.equal(r2.view(torch.int32), r2_ref.view(torch.int32))
    return float(r_ref.abs().max())


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_noalloc_matches_rhs_two_calls(prec):
    need_gpu()
    import torch
    from paper_2207_08500_amd import native
    native.load()
    P = trained_params()
    p = {"bf16": native.BF16, "fp16": native.FP16}[prec]
    margin = {"bf16": 0.5, "fp16": 0.25}[prec]
    big = inputs.uneven_sizes(inputs.BASE_SEED + 7, 300, 64, 4096)
    small = np.array([7, 300, 64, 1, 1000, 63, 65])
    qa, oa, da = _batch(inputs.BASE_SEED + 1, big)
    qb, ob, db = _batch(inputs.BASE_SEED + 2, small)
    print("no-alloc %s: %d problems / %d cells, then %d / %d"
          % (prec, big.size, int(oa[-1]), small.size, int(ob[-1])), flush=True)
    assert _compare(native, torch, P, p, margin, qa, oa, da) > 0
    assert _compare(native, torch, P, p, margin, qb, ob, db) > 0
    # a flagged "map kept" call after the smaller batch still rebuilds the map
    _compare(native, torch, P, p, margin, qa, oa, da, keep_map=True)


def test_noalloc_refuses_beyond_capacity_and_other_paths():
    need_gpu()
    import torch
    from paper_2207_08500_amd import native
    native.load()
    d = torch.device("cuda:0")
    mlp = native.Mlp(torch.as_tensor(trained_params(), device=d), recheck_margin=0.5)
    # one problem of exactly the capacity in cells: cells + 1 faces is one too many
    n = native.NOALLOC_MAX_FACES
    off = np.array([0, n], np.int64)
    prob = native.Problem(native.EULER1D, native.BF16, native.SEL_MLP, native.TRANSMISSIVE, off,
                          1.0 / n, device=d)
    q = torch.ones(3 * n, dtype=torch.float32, device=d)
    r = torch.full_like(q, 7.0)
    with pytest.raises(native.Neno6Error, match=r"\(-7\)"):
        native.neno6_rhs_noalloc(prob, mlp, q, r)
    torch.cuda.synchronize()
    assert bool((r == 7.0).all())  # nothing was enqueued
    del q, r
    # the largest accepted batch: capacity - 1 cells in one problem
    off = np.array([0, n - 1], np.int64)
    prob = native.Problem(native.EULER1D, native.BF16, native.SEL_MLP, native.TRANSMISSIVE, off,
                          1.0 / (n - 1), device=d)
    rho = np.where(np.arange(n - 1) < (n - 1) // 2, 1.0, 0.125)
    pr = np.where(np.arange(n - 1) < (n - 1) // 2, 1.0, 0.1)
    qh = inputs.conservative1d(rho, np.zeros(n - 1), pr, 1.4)
    q = torch.as_tensor(qh, dtype=torch.float32, device=d).contiguous()
    r = torch.full_like(q, float("nan"))
    native.neno6_rhs_noalloc(prob, mlp, q, r)
    r_ref = torch.zeros_like(q)
    native.neno6_rhs(prob, mlp, q, r_ref, prob.workspace(d))
    torch.cuda.synchronize()
    assert torch.equal(r.view(torch.int32), r_ref.view(torch.int32))
    del q, r, r_ref
    # FP64 and 2D go through neno6_rhs only
    off = np.array([0, 16], np.int64)
    p64 = native.Problem(native.EULER1D, native.FP64, native.SEL_MLP, native.TRANSMISSIVE, off,
                         1.0 / 16, device=d)
    q64 = torch.ones(48, dtype=torch.float64, device=d)
    with pytest.raises(native.Neno6Error, match=r"\(-5\)"):
        native.neno6_rhs_noalloc(p64, native.Mlp(torch.as_tensor(trained_params(), device=d)),
                                 q64, torch.zeros_like(q64))
