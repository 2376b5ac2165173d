"""The 2D sweep kernels as shipped (classifier on MFMA, re-check inside the
tile, FP16 and BF16 operands) against the FP64 oracle, element by
element: on ragged grids whose 64-face tiles cross row ends, on the
four-quadrant data with density waves and on a state the oracle advanced a
few steps.  Labels: flip rate bound, and with every evaluation re-checked
the re-checked labels.  Values: at every cell whose four faces carry the oracle's
labels, the right-hand side equals the one computed with the oracle's labels
imposed (same FP32 arithmetic after the labels) and lies within FP32
rounding of the oracle's (Alg. 2, dimension by dimension as in Sec. 4.4)."""
import numpy as np
import pytest

import oracle
from paper_2207_08500_amd import inputs
from tests._helpers import dev, host, label_flip_rate, need_gpu, stated_margins, trained_params

pytestmark = pytest.mark.gpu

MARGIN = stated_margins()


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    import torch
    from paper_2207_08500_amd import native
    native.load()
    return native, torch, trained_params()


def _states():
    yield "quadrants 67x45", inputs.riemann2d(41, 67, 45)
    yield "quadrants 130x3", inputs.riemann2d(42, 130, 3)
    yield "quadrants 64x64", inputs.riemann2d(43, 64, 64)
    q = inputs.riemann2d(44, 96, 80)
    qe, _, st = oracle.euler2d_step(q, 1 / 96, 1 / 80, 0.4, 8, 1.4, 1, trained_params(),
                                    oracle.SEL_MLP)
    assert st == 0
    yield "evolved 96x80, 8 steps", qe


def _cells_with_oracle_labels(mx, my, mx_o, my_o):
    sx = np.all(mx == mx_o, axis=0)  # [ny][nx+1] x faces with every field's label equal
    sy = np.all(my == my_o, axis=0)  # [ny+1][nx]
    return sx[:, :-1] & sx[:, 1:] & sy[:-1, :] & sy[1:, :]


@pytest.mark.parametrize("prec,mode", [(3, 0), (3, 1), (2, 0)])
@pytest.mark.parametrize("margin", ["stated", "all"])
def test_rhs2d_elementwise_against_oracle(ctx, prec, mode, margin):
    native, torch, P = ctx
    mu = MARGIN[prec] if margin == "stated" else 1e30
    for name, q in _states():
        _, ny, nx = q.shape
        q32 = q.astype(np.float32).astype(np.float64)
        r_o, mx_o, my_o, _ = oracle.euler2d_rhs(q32, 1 / nx, 1 / ny, 1.4, 1, P, oracle.SEL_MLP)
        mlp = native.Mlp(dev(P), recheck_margin=mu, recheck_mode=mode)
        prob = native.Problem(native.EULER2D, prec, native.SEL_MLP, 1, nx=nx, ny=ny, dx2d=1 / nx,
                              dy2d=1 / ny)
        qg = dev(q32, torch.float32)
        r = torch.zeros_like(qg)
        m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
        native.neno6_rhs(prob, mlp, qg, r, prob.workspace(), masks_out=m)
        # the same pass with the oracle's labels imposed
        mo = np.concatenate([mx_o.ravel(), my_o.ravel()])
        pin = native.Problem(native.EULER2D, prec, native.SEL_MASKS_IN, 1, nx=nx, ny=ny,
                             dx2d=1 / nx, dy2d=1 / ny)
        r_in = torch.zeros_like(qg)
        native.neno6_rhs(pin, mlp, qg, r_in, pin.workspace(), masks_in=dev(mo))
        torch.cuda.synchronize()
        m = host(m)
        nfx = 4 * (nx + 1) * ny
        mx, my = m[:nfx].reshape(4, ny, nx + 1), m[nfx:].reshape(4, ny + 1, nx)
        flips = label_flip_rate(m, mo)
        ok = _cells_with_oracle_labels(mx, my, mx_o, my_o)
        r, r_in = host(r).reshape(q.shape), host(r_in).reshape(q.shape)
        fscale = np.abs(r_o).max() + np.abs(q).max() * max(nx, ny)
        err = np.abs(r - r_o)[:, ok].max() / fscale
        same = np.array_equal(r[:, ok].view(np.uint32), r_in[:, ok].view(np.uint32))
        print("%s prec %d mode %d margin %s: flip rate %.3g, %.4f of the cells with oracle labels, max "
              "rel err %.3g, bitwise equal to the imposed-label pass: %s"
              % (name, prec, mode, margin, flips, ok.mean(), err, same))
        assert flips < (2e-4 if margin == "all" else 2e-3)
        assert ok.mean() > 0.98
        assert same
        assert err <= 5e-5


@pytest.mark.parametrize("prec", [2, 3])
def test_rhs2d_masks_in_every_selection(ctx, prec):
    """Imposed labels drawn at random (all 256 selection pairs occur in both
    sweeps): the sweep's combine, one coefficient stencil per selection,
    matches the oracle's re-normalised combination to FP32 rounding."""
    native, torch, P = ctx
    q = inputs.riemann2d(45, 67, 45)
    _, ny, nx = q.shape
    q32 = q.astype(np.float32).astype(np.float64)
    nm = 4 * ((nx + 1) * ny + nx * (ny + 1))
    mi = np.random.default_rng(46).integers(0, 256, nm).astype(np.uint8)
    assert len(np.unique(mi)) == 256
    nfx = 4 * (nx + 1) * ny
    r_o, mx_o, my_o, _ = oracle.euler2d_rhs(q32, 1 / nx, 1 / ny, 1.4, 1, P, oracle.SEL_MASKS_IN,
                                             masks_in=(mi[:nfx], mi[nfx:]))
    assert np.array_equal(np.concatenate([mx_o.ravel(), my_o.ravel()]), mi)
    mlp = native.Mlp(dev(P), recheck_margin=MARGIN[prec])
    pin = native.Problem(native.EULER2D, prec, native.SEL_MASKS_IN, 1, nx=nx, ny=ny, dx2d=1 / nx,
                         dy2d=1 / ny)
    qg = dev(q32, torch.float32)
    r = torch.zeros_like(qg)
    native.neno6_rhs(pin, mlp, qg, r, pin.workspace(), masks_in=dev(mi))
    torch.cuda.synchronize()
    r = host(r).reshape(q.shape)
    fscale = np.abs(r_o).max() + np.abs(q).max() * max(nx, ny)
    err = np.abs(r - r_o).max() / fscale
    print("prec %d: max rel err %.3g" % (prec, err))
    assert err <= 5e-5
