"""Reduced-precision paths (FP32 vector, BF16/FP16 MFMA with the FP32
re-check) against the FP64 oracle on identical inputs.  Labels are compared
as flip rates with stated bounds; values with the oracle's selection imposed
(so only the arithmetic precision differs) to FP32-level tolerances."""
import numpy as np
import pytest

import oracle
from paper_2207_08500_amd import inputs
from tests._helpers import dev, host, label_flip_rate, need_gpu, trained_params, stated_margins

pytestmark = pytest.mark.gpu

# Re-check margins (logit units) of the committed weights: twice the largest
# reduced-precision logit error observed on 2^20 classifier-training samples
# (tests/test_gpu_margin.py re-derives them).
MARGIN = stated_margins()


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    import torch
    from paper_2207_08500_amd import native
    P = trained_params()
    return native, torch, P


def _mlp(native, P, prec, mode=0):
    return native.Mlp(dev(P), recheck_margin=MARGIN.get(prec, 0.0), recheck_mode=mode)


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_logits_against_oracle(ctx, prec):
    native, torch, P = ctx
    n = 1 << 16
    s, _ = inputs.classifier_samples(20, n)
    _, z_o = oracle.mlp_logits(P, s)
    mlp = _mlp(native, P, prec)
    z = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    m = torch.zeros(n, dtype=torch.uint8, device="cuda")
    native.neno6_mlp_logits(mlp, prec, dev(s, torch.float32), z, m)
    torch.cuda.synchronize()
    z, m = host(z), host(m)
    err = np.abs(z - z_o)
    want = sum(((z_o[:, k] <= 0).astype(np.uint8) << k) for k in range(4))
    flips = label_flip_rate(m, want, ("lo",))
    print("prec %d: max |dz| %.3g, label flip rate %.3g" % (prec, err.max(), flips))
    if prec == 1:
        assert err.max() <= 1e-4 * max(1.0, np.abs(z_o).max())
        # FP32 labels differ from FP64 only for logits within round-off of 0
        bad = (m != want)
        assert np.all(np.abs(z_o[bad]).min(axis=1) < 1e-3)
    else:
        # the margin is twice the largest error on another 2^20 samples of
        # this distribution: these samples' errors stay within it
        assert err.max() < MARGIN[prec]
        # labels: an evaluation beyond the margin keeps the reduced-precision
        # label, which must be the FP64 one; one within it takes the
        # re-check's label, which differs from FP64 only within the re-check's
        # rounding of the cutoff.  So every differing label has an FP64 logit
        # at 0.
        bad = m != want
        assert np.all(np.abs(z_o[bad]).min(axis=1) < 1e-3)
        assert flips < 1e-5


@pytest.mark.parametrize("prec,mode", [(2, 0), (3, 0), (3, 1)])
def test_recheck_logits_against_oracle(ctx, prec, mode):
    """With every evaluation inside the margin the logits are the re-check's:
    FP32 on the vector units (the default re-check arithmetic), held to the
    FP32 mode's bound; with the two-part FP16 re-check (FP16 operands;
    weights and activations each as an FP16 value plus the FP16 rounding of
    the remainder, FP32 sums), whose operands carry 21-22 significant bits
    against FP32's 24: held to eight times that bound.  The labels are the signs of these logits, and a
    label differs from FP64 only for a logit within 1e-3 of the cutoff."""
    native, torch, P = ctx
    n = 1 << 16
    s, _ = inputs.classifier_samples(20, n)
    s32 = s.astype(np.float32).astype(np.float64)
    _, z_o = oracle.mlp_logits(P, s32)
    mlp = native.Mlp(dev(P), recheck_margin=1e30, recheck_mode=mode)
    z = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    m = torch.zeros(n, dtype=torch.uint8, device="cuda")
    native.neno6_mlp_logits(mlp, prec, dev(s32, torch.float32), z, m)
    torch.cuda.synchronize()
    z, m = host(z).astype(np.float64), host(m)
    err = np.abs(z - z_o)
    scale = max(1.0, np.abs(z_o).max())
    print("prec %d mode %d, every evaluation re-checked: max |dz| %.3g (%.3g of the largest "
          "logit), median %.3g" % (prec, mode, err.max(), err.max() / scale, np.median(err)))
    assert np.array_equal(m, sum(((z[:, k] <= 0).astype(np.uint8) << k) for k in range(4)))
    assert err.max() <= (8e-4 if mode == native.RECHECK_FP16X2 else 1e-4) * scale
    want = sum(((z_o[:, k] <= 0).astype(np.uint8) << k) for k in range(4))
    bad = m != want
    assert np.all(np.abs(z_o[bad]).min(axis=1) < 1e-3)


@pytest.mark.parametrize("prec,mode", [(1, 0), (2, 0), (3, 0), (3, 1)])
@pytest.mark.parametrize("sign", [1, -1])
def test_reconstruct_against_oracle(ctx, prec, mode, sign):
    native, torch, P = ctx
    n = 3001
    f = inputs.random_stencils(21, (n + 10) // 6 + 1).ravel()[: n + 5]
    fh_o, m_o = oracle.reconstruct(f, sign, P, oracle.SEL_MLP)
    mlp = _mlp(native, P, prec, mode)
    fh = torch.zeros(n, dtype=torch.float32, device="cuda")
    m = torch.zeros(n, dtype=torch.uint8, device="cuda")
    native.neno6_reconstruct(mlp, dev(f, torch.float32), sign, prec, native.SEL_MLP, fh, masks_out=m)
    # the same selection imposed: only the FP32 arithmetic differs
    fh2 = torch.zeros(n, dtype=torch.float32, device="cuda")
    native.neno6_reconstruct(mlp, dev(f, torch.float32), sign, prec, native.SEL_MASKS_IN, fh2,
                             masks_in=dev(m_o))
    torch.cuda.synchronize()
    assert label_flip_rate(host(m), m_o, ("lo",)) < 2e-3
    scale = np.abs(f).reshape(-1)[: n + 5]
    loc = np.maximum.reduce([np.abs(f[j:j + n]) for j in range(6)])
    assert np.all(np.abs(host(fh2) - fh_o) <= 1e-5 * np.maximum(loc, 1e-30) * 4)


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_euler1d_rhs_against_oracle(ctx, prec):
    native, torch, P = ctx
    sizes = (1, 2, 7, 64, 65, 500, 1000)
    q, off, dx = inputs.riemann1d_batch(22, sizes, perturb=True)
    r_o, m_o, _ = oracle.euler1d_rhs(q, off, dx, 1.4, 1, P, oracle.SEL_MLP)
    mlp = _mlp(native, P, prec)
    prob = native.Problem(native.EULER1D, prec, native.SEL_MLP, 1, off, dx)
    qg = dev(q, torch.float32)
    ws = prob.workspace()
    r = torch.zeros_like(qg)
    m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
    native.neno6_rhs(prob, mlp, qg, r, ws, masks_out=m)
    prob_in = native.Problem(native.EULER1D, prec, native.SEL_MASKS_IN, 1, off, dx)
    r2 = torch.zeros_like(qg)
    native.neno6_rhs(prob_in, mlp, qg, r2, prob_in.workspace(), masks_in=dev(m_o.ravel()))
    torch.cuda.synchronize()
    flips = label_flip_rate(host(m), m_o.ravel())
    print("prec %d euler1d flip rate %.3g" % (prec, flips))
    assert flips < 2e-3
    # values with the oracle's selection: FP32 rounding of the state and the
    # arithmetic, relative to the size of the fluxes in each line
    r2 = host(r2).reshape(3, -1)
    for p in range(len(sizes)):
        a, b = off[p], off[p + 1]
        fscale = np.abs(r_o[:, a:b]).max() + np.abs(q[:, a:b]).max() / dx[p]
        assert np.abs(r2[:, a:b] - r_o[:, a:b]).max() <= 5e-5 * fscale


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_euler2d_rhs_against_oracle(ctx, prec):
    native, torch, P = ctx
    nx, ny = 67, 45
    q = inputs.riemann2d(23, nx, ny)
    r_o, mx_o, my_o, _ = oracle.euler2d_rhs(q, 1 / nx, 1 / ny, 1.4, 1, P, oracle.SEL_MLP)
    mlp = _mlp(native, P, prec)
    prob = native.Problem(native.EULER2D, prec, native.SEL_MLP, 1, nx=nx, ny=ny, dx2d=1 / nx, dy2d=1 / ny)
    qg = dev(q, torch.float32)
    r = torch.zeros_like(qg)
    m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
    native.neno6_rhs(prob, mlp, qg, r, prob.workspace(), masks_out=m)
    prob_in = native.Problem(native.EULER2D, prec, native.SEL_MASKS_IN, 1, nx=nx, ny=ny,
                             dx2d=1 / nx, dy2d=1 / ny)
    r2 = torch.zeros_like(qg)
    mo = np.concatenate([mx_o.ravel(), my_o.ravel()])
    native.neno6_rhs(prob_in, mlp, qg, r2, prob_in.workspace(), masks_in=dev(mo))
    torch.cuda.synchronize()
    flips = label_flip_rate(host(m), mo)
    print("prec %d euler2d flip rate %.3g" % (prec, flips))
    assert flips < 2e-3
    fscale = np.abs(r_o).max() + np.abs(q).max() * max(nx, ny)
    assert np.abs(host(r2).reshape(q.shape) - r_o).max() <= 5e-5 * fscale


@pytest.mark.parametrize("prec,mode", [(2, 0), (3, 0), (3, 1)])
@pytest.mark.parametrize("nx,ny", [(67, 45), (130, 3)])
def test_euler2d_recheck_lists_complete(ctx, prec, mode, nx, ny):
    """With a margin that every logit falls inside, the 2D re-check lists
    hold every evaluation of both sweeps (eight per face, ragged grids), and
    the labels then come from the re-check (FP32 or two-part FP16): a flip
    rate at the re-check's rounding level against the FP64 oracle.  Margin 0 queues nothing."""
    native, torch, P = ctx
    q = inputs.riemann2d(29, nx, ny)
    _, mx_o, my_o, _ = oracle.euler2d_rhs(q, 1 / nx, 1 / ny, 1.4, 1, P, oracle.SEL_MLP)
    mo = np.concatenate([mx_o.ravel(), my_o.ravel()])
    nfx, nfy = (nx + 1) * ny, nx * (ny + 1)
    qg = dev(q, torch.float32)
    for margin in (0.0, 1e30):
        mlp = native.Mlp(dev(P), recheck_margin=margin, recheck_mode=mode)
        prob = native.Problem(native.EULER2D, prec, native.SEL_MLP, 1, nx=nx, ny=ny, dx2d=1 / nx,
                              dy2d=1 / ny)
        ws = prob.workspace()
        F = torch.zeros(4 * (nfx + nfy), dtype=torch.float32, device="cuda")
        m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
        native.neno6_face_fluxes(prob, mlp, qg, F, ws, masks_out=m)
        cnt = native.neno6_recheck_count(prob, mlp, ws)
        assert cnt == ((0, 0) if margin == 0.0 else (8 * nfx, 8 * nfy))
        if margin > 0.0:
            flips = label_flip_rate(host(m), mo)
            print("prec %d %dx%d all re-checked: flip rate %.3g" % (prec, nx, ny, flips))
            assert flips < 1e-3


@pytest.mark.parametrize("prec", [2, 3])
def test_euler1d_steps_error(ctx, prec):
    """Twenty RK3 steps of a 1D Euler batch against the FP64 oracle run."""
    native, torch, P = ctx
    sizes = (256, 400, 1000)
    q, off, dx = inputs.riemann1d_batch(24, sizes, perturb=True)
    q_o, t_o, st_o = oracle.euler1d_step(q, off, dx, 0.4, 20, 1.4, 1, P, oracle.SEL_MLP)
    mlp = _mlp(native, P, prec)
    prob = native.Problem(native.EULER1D, prec, native.SEL_MLP, 1, off, dx)
    qg = dev(q, torch.float32)
    t = torch.zeros(len(sizes), dtype=torch.float64, device="cuda")
    st = torch.zeros(len(sizes), dtype=torch.int32, device="cuda")
    native.neno6_step(prob, mlp, qg, 0.4, 20, t, st, prob.workspace())
    torch.cuda.synchronize()
    qf = host(qg).reshape(3, -1)
    assert np.array_equal(host(st), st_o)
    for p in range(len(sizes)):
        a, b = off[p], off[p + 1]
        l1 = np.abs(qf[:, a:b] - q_o[:, a:b]).mean(axis=1) / np.abs(q_o[:, a:b]).mean(axis=1)
        print("prec %d problem %d relative L1 %s" % (prec, p, l1))
        # FP32 state rounding over 20 steps (a few 1e-7 relative per step);
        # a label flipped near a shock would move a few cells by O(1e-3) of
        # the jump, about 1e-5 of the L1 norm of a 256-cell line
        assert np.all(l1 < 1e-4)
    # the CFL step follows the largest wave speed of the (FP32-rounded) state
    assert np.allclose(host(t), t_o, rtol=1e-5)


@pytest.mark.parametrize("prec", [2, 3])
def test_c2_full_size_sampled(ctx, prec):
    """The benchmark's 256 x 4000-cell batch in the benchmark's configuration
    (FP32 state, autotuned launch shape, re-check on): labels against the
    oracle's on the same (FP32-rounded) state for sampled problems, and the
    right-hand side with the oracle's labels imposed within FP32 rounding."""
    native, torch, P = ctx
    from paper_2207_08500_amd import autotune
    q, off, dx = inputs.riemann1d_batch(inputs.BASE_SEED, (4000,) * 256)
    q32 = q.astype(np.float32).astype(np.float64)
    mlp = _mlp(native, P, prec)
    prob = native.Problem(native.EULER1D, prec, native.SEL_MLP, 1, off, dx)
    qg = dev(q32, torch.float32)
    ws = prob.workspace()
    autotune.tuned(prob, mlp, qg, ws)
    r = torch.zeros_like(qg)
    m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
    native.neno6_rhs(prob, mlp, qg, r, ws, masks_out=m)
    torch.cuda.synchronize()
    r, m = host(r).reshape(3, -1), host(m).reshape(3, -1)
    flips = []
    for p in (0, 41, 128, 200, 255):
        a, b = off[p], off[p + 1]
        sub = q32[:, a:b]
        r_o, m_o, _ = oracle.euler1d_rhs(sub, [0, 4000], dx[p:p + 1], 1.4, 1, P, oracle.SEL_MLP)
        flips.append(label_flip_rate(m[:, a + p:b + p + 1].ravel(), m_o.ravel()))
        # the same labels imposed: only FP32 arithmetic differs
        prob_in = native.Problem(native.EULER1D, prec, native.SEL_MASKS_IN, 1, [0, 4000], dx[p:p + 1])
        r2 = torch.zeros(3 * 4000, dtype=torch.float32, device="cuda")
        native.neno6_rhs(prob_in, mlp, dev(sub, torch.float32), r2, prob_in.workspace(),
                         masks_in=dev(m_o.ravel()))
        torch.cuda.synchronize()
        fscale = np.abs(r_o).max() + np.abs(sub).max() / dx[p]
        assert np.abs(host(r2).reshape(3, -1) - r_o).max() <= 5e-5 * fscale
    print("C2 prec %d: sampled label flip rates %s" % (prec, flips))
    assert max(flips) < 1e-4
