"""FP64 path against the FP64 oracle: classification labels, face values,
right-hand sides and time steps must be identical bit for bit (the GPU path
evaluates the same operations in the same order, without FP contraction).
All calls go through the C ABI (libneno6.so)."""
import numpy as np
import pytest

import oracle
from paper_2207_08500_amd import inputs
from tests._helpers import dev, host, need_gpu, trained_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    import torch
    from paper_2207_08500_amd import native
    P = trained_params()
    mlp = native.Mlp(dev(P), recheck_margin=0.0)
    return native, torch, P, mlp


def _same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape
    bad = ~((a == b) | (np.isnan(a) & np.isnan(b)))
    assert not bad.any(), "first mismatch at %s: %r vs %r (%d of %d differ)" % (
        np.argwhere(bad)[0], a[bad][0], b[bad][0], bad.sum(), bad.size)


@pytest.mark.parametrize("n_faces", [1, 63, 64, 65, 1000, 4099])
@pytest.mark.parametrize("sign", [1, -1])
def test_reconstruct_mlp_bitwise(ctx, n_faces, sign):
    native, torch, P, mlp = ctx
    f = inputs.random_stencils(100 + n_faces, (n_faces + 5 + 5) // 6 + 1).ravel()[: n_faces + 5]
    fh_o, m_o = oracle.reconstruct(f, sign, P, oracle.SEL_MLP)
    fh = torch.zeros(n_faces, dtype=torch.float64, device="cuda")
    m = torch.zeros(n_faces, dtype=torch.uint8, device="cuda")
    native.neno6_reconstruct(mlp, dev(f), sign, native.FP64, native.SEL_MLP, fh, masks_out=m)
    torch.cuda.synchronize()
    _same(host(m), m_o)
    _same(host(fh), fh_o)


@pytest.mark.parametrize("selector", [1, 2, 3])
def test_reconstruct_selectors_bitwise(ctx, selector):
    native, torch, P, mlp = ctx
    n = 777
    f = inputs.random_stencils(7, 140).ravel()[: n + 5]
    mi = np.random.default_rng(0).integers(0, 16, n).astype(np.uint8)
    fh_o, m_o = oracle.reconstruct(f, 1, None, selector, mi)
    fh = torch.zeros(n, dtype=torch.float64, device="cuda")
    m = torch.zeros(n, dtype=torch.uint8, device="cuda")
    native.neno6_reconstruct(None, dev(f), 1, native.FP64, selector, fh, masks_in=dev(mi), masks_out=m)
    torch.cuda.synchronize()
    _same(host(m), m_o)
    _same(host(fh), fh_o)


def test_logits_bitwise(ctx):
    native, torch, P, mlp = ctx
    s, _ = inputs.classifier_samples(8, 5000)
    _, z_o = oracle.mlp_logits(P, s)
    z = torch.zeros((5000, 4), dtype=torch.float64, device="cuda")
    m = torch.zeros(5000, dtype=torch.uint8, device="cuda")
    native.neno6_mlp_logits(mlp, native.FP64, dev(s), z, m)
    torch.cuda.synchronize()
    _same(host(z), z_o)
    want = sum(((z_o[:, k] <= 0).astype(np.uint8) << k) for k in range(4))
    _same(host(m), want)


def _run_rhs(native, torch, mlp, prob, q, masks_in=None):
    nb = prob.mask_count()
    r = torch.zeros_like(q)
    m = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    st = torch.zeros(prob.n_problems, dtype=torch.int32, device="cuda")
    ws = prob.workspace()
    native.neno6_rhs(prob, mlp, q, r, ws, masks_in=masks_in, masks_out=m, status=st)
    torch.cuda.synchronize()
    return host(r), host(m), host(st)


@pytest.mark.parametrize("bc", [0, 1])
def test_advection_rhs_bitwise(ctx, bc):
    native, torch, P, mlp = ctx
    u = inputs.advection_c1(9, 200)
    dx = 2.0 / 200
    r_o, m_o = oracle.advection_rhs(u, dx, bc, P, oracle.SEL_MLP)
    prob = native.Problem(native.ADVECTION, native.FP64, native.SEL_MLP, bc, [0, 200], [dx])
    r, m, _ = _run_rhs(native, torch, mlp, prob, dev(u))
    _same(m, m_o)
    _same(r, r_o)


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("selector", [0, 1, 2, 3])
def test_euler1d_rhs_bitwise(ctx, bc, selector):
    native, torch, P, mlp = ctx
    sizes = (1, 2, 3, 7, 64, 65, 200, 333)
    q, off, dx = inputs.riemann1d_batch(10 + selector, sizes, perturb=True)
    tf = int(off[-1]) + len(sizes)
    mi = np.random.default_rng(1).integers(0, 256, (3, tf)).astype(np.uint8)
    r_o, m_o, st_o = oracle.euler1d_rhs(q, off, dx, 1.4, bc, P, selector, mi)
    prob = native.Problem(native.EULER1D, native.FP64, selector, bc, off, dx)
    r, m, st = _run_rhs(native, torch, mlp, prob, dev(q), masks_in=dev(mi))
    _same(st, st_o)
    _same(m.reshape(3, -1), m_o)
    _same(r.reshape(3, -1), r_o)


@pytest.mark.parametrize("bc", [0, 1])
def test_euler2d_rhs_bitwise(ctx, bc):
    native, torch, P, mlp = ctx
    q = inputs.riemann2d(11, 37, 29)
    r_o, mx_o, my_o, st_o = oracle.euler2d_rhs(q, 1 / 37, 1 / 29, 1.4, bc, P, oracle.SEL_MLP)
    prob = native.Problem(native.EULER2D, native.FP64, native.SEL_MLP, bc, nx=37, ny=29,
                          dx2d=1 / 37, dy2d=1 / 29)
    r, m, st = _run_rhs(native, torch, mlp, prob, dev(q))
    nfx = 4 * 38 * 29
    _same(m[:nfx].reshape(mx_o.shape), mx_o)
    _same(m[nfx:].reshape(my_o.shape), my_o)
    _same(r.reshape(q.shape), r_o)
    assert st[0] == st_o[0]


def test_advection_c1_full_run_bitwise(ctx):
    """The whole C1 case (N = 200, CFL 0.4, t = 2: 500 RK3 steps)."""
    native, torch, P, mlp = ctx
    u = inputs.advection_c1(inputs.BASE_SEED, 200)
    dx = 2.0 / 200
    u_o = oracle.advection_step(u, dx, 0.4 * dx, 500, oracle.BC_PERIODIC, P, oracle.SEL_MLP)
    prob = native.Problem(native.ADVECTION, native.FP64, native.SEL_MLP, native.PERIODIC, [0, 200], [dx])
    ug = dev(u)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    native.neno6_step(prob, mlp, ug, 0.4, 500, t, st, prob.workspace())
    torch.cuda.synchronize()
    _same(host(ug), u_o)
    assert abs(host(t)[0] - 2.0) < 1e-12


@pytest.mark.parametrize("bc", [0, 1])
def test_euler1d_steps_bitwise(ctx, bc):
    native, torch, P, mlp = ctx
    sizes = (5, 40, 64, 129, 300)
    q, off, dx = inputs.riemann1d_batch(12, sizes, perturb=True)
    q_o, t_o, st_o = oracle.euler1d_step(q, off, dx, 0.4, 6, 1.4, bc, P, oracle.SEL_MLP)
    prob = native.Problem(native.EULER1D, native.FP64, native.SEL_MLP, bc, off, dx)
    qg = dev(q)
    t = torch.zeros(len(sizes), dtype=torch.float64, device="cuda")
    st = torch.zeros(len(sizes), dtype=torch.int32, device="cuda")
    native.neno6_step(prob, mlp, qg, 0.4, 6, t, st, prob.workspace())
    torch.cuda.synchronize()
    _same(host(st), st_o)
    _same(host(t), t_o)
    _same(host(qg).reshape(3, -1), q_o)


def test_euler1d_nonphysical_freeze(ctx):
    native, torch, P, mlp = ctx
    q, off, dx = inputs.riemann1d_batch(13, (30, 30, 30), perturb=True)
    q[2, 45] = -1.0  # negative energy in problem 1
    q_o, t_o, st_o = oracle.euler1d_step(q, off, dx, 0.4, 3, 1.4, 1, P, oracle.SEL_ALL_DISCARD)
    assert list(st_o) == [0, -4, 0]
    prob = native.Problem(native.EULER1D, native.FP64, native.SEL_ALL_DISCARD, 1, off, dx)
    qg = dev(q)
    t = torch.zeros(3, dtype=torch.float64, device="cuda")
    st = torch.zeros(3, dtype=torch.int32, device="cuda")
    native.neno6_step(prob, mlp, qg, 0.4, 3, t, st, prob.workspace())
    torch.cuda.synchronize()
    _same(host(st), st_o)
    _same(host(t), t_o)
    _same(host(qg).reshape(3, -1), q_o)


def test_euler2d_steps_bitwise(ctx):
    native, torch, P, mlp = ctx
    q = inputs.riemann2d(14, 24, 20)
    q_o, t_o, st_o = oracle.euler2d_step(q, 1 / 24, 1 / 20, 0.4, 3, 1.4, 1, P, oracle.SEL_MLP)
    prob = native.Problem(native.EULER2D, native.FP64, native.SEL_MLP, 1, nx=24, ny=20,
                          dx2d=1 / 24, dy2d=1 / 20)
    qg = dev(q)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    native.neno6_step(prob, mlp, qg, 0.4, 3, t, st, prob.workspace())
    torch.cuda.synchronize()
    assert host(st)[0] == st_o
    assert host(t)[0] == t_o
    _same(host(qg).reshape(q.shape), q_o)


def test_c2_full_size_sampled_bitwise(ctx):
    """The 256 x 4000-cell 1D Euler batch in FP64: the GPU right-hand side of
    the whole batch against the oracle on a sample of its problems (problems
    are independent, so a sub-batch gives the same values)."""
    native, torch, P, mlp = ctx
    q, off, dx = inputs.riemann1d_batch(inputs.BASE_SEED, (4000,) * 256)
    prob = native.Problem(native.EULER1D, native.FP64, native.SEL_MLP, 1, off, dx)
    r, m, st = _run_rhs(native, torch, mlp, prob, dev(q))
    r = r.reshape(3, -1)
    m = m.reshape(3, -1)
    for p in (0, 97, 255):
        sub = q[:, off[p]:off[p + 1]]
        r_o, m_o, st_o = oracle.euler1d_rhs(sub, [0, 4000], dx[p:p + 1], 1.4, 1, P, oracle.SEL_MLP)
        _same(r[:, off[p]:off[p + 1]], r_o)
        _same(m[:, off[p] + p:off[p + 1] + p + 1], m_o)
        assert st[p] == st_o[0]


def test_c3_full_size_sampled_bitwise(ctx):
    """The 2048 x 2048 2D Euler grid in FP64: sampled cells against the oracle
    on a window around each (a cell's right-hand side only reads three cells
    along its row and column, so the window gives the exact value)."""
    native, torch, P, mlp = ctx
    n = 2048
    q = inputs.riemann2d(inputs.BASE_SEED, n, n)
    prob = native.Problem(native.EULER2D, native.FP64, native.SEL_MLP, 1, nx=n, ny=n,
                          dx2d=1 / n, dy2d=1 / n)
    qg = dev(q)
    r = torch.zeros_like(qg)
    native.neno6_rhs(prob, mlp, qg, r, prob.workspace())
    torch.cuda.synchronize()
    r = host(r)
    rng = np.random.default_rng(5)
    pts = [(0, 0), (n - 1, n - 1), (1023, 1024), (2, n - 3)] + [tuple(rng.integers(0, n, 2)) for _ in range(8)]
    for (y0, x0) in pts:
        ya, yb = max(0, y0 - 3), min(n, y0 + 4)
        xa, xb = max(0, x0 - 3), min(n, x0 + 4)
        win = q[:, ya:yb, xa:xb]
        r_o, _, _, _ = oracle.euler2d_rhs(win, 1 / n, 1 / n, 1.4, 1, P, oracle.SEL_MLP)
        _same(r[:, y0, x0], r_o[:, y0 - ya, x0 - xa])
