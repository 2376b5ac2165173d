"""Batches of 2D grids of uneven sizes in one call (Sec. 4.4, dimension by
dimension on each grid): the FP64 path against the oracle grid by grid, bit
for bit (labels, right-hand sides, steps with each grid's own time step);
the reduced-precision paths (FP32 and two-part FP16 re-checks) against the
same calls made grid by grid; a HIP-graph replay of a batched step; face
fluxes and the vector-Jacobian product of a batch."""
import numpy as np
import pytest

import oracle
from paper_2207_08500_amd import inputs
from tests._helpers import dev, host, need_gpu, stated_margins, trained_params

pytestmark = pytest.mark.gpu

MARGIN = stated_margins()
SIZES = [(67, 45), (130, 3), (64, 64), (5, 97)]


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    import torch
    from paper_2207_08500_amd import native
    native.load()
    grids = [(nx, ny, 1.0 / nx, 1.0 / ny) for nx, ny in SIZES]
    qs = [inputs.riemann2d(60 + i, nx, ny) for i, (nx, ny) in enumerate(SIZES)]
    return native, torch, trained_params(), grids, qs


def _batch(native, prec, grids):
    return native.Problem(native.EULER2D, prec, native.SEL_MLP, 1, grids=grids)


def _single(native, prec, g):
    nx, ny, dx, dy = g
    return native.Problem(native.EULER2D, prec, native.SEL_MLP, 1, nx=nx, ny=ny, dx2d=dx, dy2d=dy)


def _split(arr, grids, per):
    """Pieces of a batch array, grid by grid; per(nx, ny) entries each."""
    out, o = [], 0
    for nx, ny, _, _ in grids:
        n = per(nx, ny)
        out.append(arr[o:o + n])
        o += n
    assert o == arr.size
    return out


def _cells(nx, ny):
    return 4 * nx * ny


def _faces(nx, ny):
    return 4 * ((nx + 1) * ny + nx * (ny + 1))


def test_fp64_batch_rhs_equals_oracle(ctx):
    native, torch, P, grids, qs = ctx
    prob = _batch(native, native.FP64, grids)
    mlp = native.Mlp(dev(P))
    q = dev(np.concatenate([x.ravel() for x in qs]))
    r = torch.zeros_like(q)
    m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
    native.neno6_rhs(prob, mlp, q, r, prob.workspace(), masks_out=m)
    torch.cuda.synchronize()
    rs, ms = _split(host(r), grids, _cells), _split(host(m), grids, _faces)
    for (nx, ny, dx, dy), qg, rg, mg in zip(grids, qs, rs, ms):
        r_o, mx_o, my_o, _ = oracle.euler2d_rhs(qg, dx, dy, 1.4, 1, P, oracle.SEL_MLP)
        assert np.array_equal(rg, r_o.ravel())
        assert np.array_equal(mg, np.concatenate([mx_o.ravel(), my_o.ravel()]))


def test_fp64_batch_steps_equal_oracle(ctx):
    """Each grid takes its own time step (its own CFL maximum and spacing)."""
    native, torch, P, grids, qs = ctx
    prob = _batch(native, native.FP64, grids)
    q = dev(np.concatenate([x.ravel() for x in qs]))
    n = len(grids)
    t = torch.zeros(n, dtype=torch.float64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    native.neno6_step(prob, native.Mlp(dev(P)), q, 0.4, 3, t, st, prob.workspace())
    torch.cuda.synchronize()
    qs_out, t, st = _split(host(q), grids, _cells), host(t), host(st)
    assert np.all(st == 0)
    for i, ((nx, ny, dx, dy), qg) in enumerate(zip(grids, qs)):
        q_o, t_o, st_o = oracle.euler2d_step(qg, dx, dy, 0.4, 3, 1.4, 1, P, oracle.SEL_MLP)
        assert st_o == 0
        assert np.array_equal(qs_out[i], q_o.ravel())
        assert t[i] == t_o
    assert len(set(t.tolist())) == n  # every grid its own time step


@pytest.mark.parametrize("prec,mode", [(3, 0), (3, 1), (2, 0)])
def test_reduced_batch_equals_grid_by_grid(ctx, prec, mode):
    """Right-hand side, labels, face fluxes and two RK3 steps of the batch are
    bitwise those of the same calls made grid by grid (same kernels, same
    launch shapes)."""
    native, torch, P, grids, qs = ctx
    mlp = native.Mlp(dev(P), recheck_margin=MARGIN[prec], recheck_mode=mode)
    prob = _batch(native, prec, grids)
    ws = prob.workspace()
    q = dev(np.concatenate([x.ravel() for x in qs]), torch.float32)
    r = torch.zeros_like(q)
    m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
    F = torch.zeros(4 * prob.n_faces, dtype=torch.float32, device="cuda")
    native.neno6_rhs(prob, mlp, q, r, ws, masks_out=m)
    native.neno6_face_fluxes(prob, mlp, q, F, ws)
    qb = q.clone()
    n = len(grids)
    t = torch.zeros(n, dtype=torch.float64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    native.neno6_step(prob, mlp, qb, 0.4, 2, t, st, ws)
    torch.cuda.synchronize()
    rs, ms = _split(host(r), grids, _cells), _split(host(m), grids, _faces)
    Fs, qbs = _split(host(F), grids, _faces), _split(host(qb), grids, _cells)
    for i, (g, qg) in enumerate(zip(grids, qs)):
        p1 = _single(native, prec, g)
        w1 = p1.workspace()
        q1 = dev(qg.ravel(), torch.float32)
        r1 = torch.zeros_like(q1)
        m1 = torch.zeros(p1.mask_count(), dtype=torch.uint8, device="cuda")
        F1 = torch.zeros(4 * p1.n_faces, dtype=torch.float32, device="cuda")
        native.neno6_rhs(p1, mlp, q1, r1, w1, masks_out=m1)
        native.neno6_face_fluxes(p1, mlp, q1, F1, w1)
        t1 = torch.zeros(1, dtype=torch.float64, device="cuda")
        s1 = torch.zeros(1, dtype=torch.int32, device="cuda")
        native.neno6_step(p1, mlp, q1, 0.4, 2, t1, s1, w1)
        torch.cuda.synchronize()
        assert np.array_equal(rs[i].view(np.uint32), host(r1).view(np.uint32))
        assert np.array_equal(ms[i], host(m1))
        assert np.array_equal(Fs[i].view(np.uint32), host(F1).view(np.uint32))
        assert np.array_equal(qbs[i].view(np.uint32), host(q1).view(np.uint32))
        assert float(host(t)[i]) == float(host(t1)[0])


def test_batch_step_graph_replay(ctx):
    """A batched FP16 step captured once and replayed three times matches
    eager steps after every replay."""
    native, torch, P, grids, qs = ctx
    mlp = native.Mlp(dev(P), recheck_margin=MARGIN[3])
    prob = _batch(native, native.FP16, grids)
    ws = prob.workspace()
    q0 = dev(np.concatenate([x.ravel() for x in qs]), torch.float32)
    n = len(grids)
    qg, tg = q0.clone(), torch.zeros(n, dtype=torch.float64, device="cuda")
    sg = torch.zeros(n, dtype=torch.int32, device="cuda")
    qe, te = q0.clone(), torch.zeros_like(tg)
    se = torch.zeros_like(sg)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        native.neno6_step(prob, mlp, qe, 0.4, 1, te, se, ws, stream=s)  # warm-up, eager
    torch.cuda.current_stream().wait_stream(s)
    qe.copy_(q0)
    te.zero_()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        native.neno6_step(prob, mlp, qg, 0.4, 1, tg, sg, ws)
    qg.copy_(q0)
    tg.zero_()
    sg.zero_()
    torch.cuda.synchronize()
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        native.neno6_step(prob, mlp, qe, 0.4, 1, te, se, ws)
        torch.cuda.synchronize()
        assert torch.equal(qg, qe) and torch.equal(tg, te) and torch.equal(sg, se)


def test_batch_vjp_equals_grid_by_grid(ctx):
    native, torch, P, grids, qs = ctx
    prob = _batch(native, native.FP64, grids)
    q = dev(np.concatenate([x.ravel() for x in qs]))
    m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device="cuda")
    native.neno6_rhs(prob, native.Mlp(dev(P)), q, torch.zeros_like(q), prob.workspace(),
                     masks_out=m)
    rbar = dev(np.random.default_rng(7).standard_normal(q.numel()))
    qbar = torch.zeros_like(q)
    native.neno6_rhs_vjp(prob, q, m, rbar, qbar)
    torch.cuda.synchronize()
    qbs = _split(host(qbar), grids, _cells)
    ms, rbs = _split(host(m), grids, _faces), _split(host(rbar), grids, _cells)
    for i, (g, qg) in enumerate(zip(grids, qs)):
        p1 = _single(native, native.FP64, g)
        qb1 = torch.zeros(qg.size, dtype=torch.float64, device="cuda")
        native.neno6_rhs_vjp(p1, dev(qg.ravel()), dev(ms[i]), dev(rbs[i]), qb1)
        torch.cuda.synchronize()
        assert np.array_equal(qbs[i], host(qb1))
