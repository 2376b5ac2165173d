"""Pins of the oracle's inviscid Burgers solver (Sec. 4.3, eq. Burgers: flux
u^2/2, Rusanov splitting, NENO6 / TENO6-opt reconstruction, SSP-RK3)
against what the mathematics fixes:

* conservation of sum(u) on periodic grids;
* before shocks form, the solution given by the characteristics,
  u = u0(x - u t), with fourth-order convergence of the optimal scheme;
* the Rankine-Hugoniot speed (uL + uR) / 2 of a shock;
* the centred rarefaction fan u = (x - x0) / t;
* the symmetry u(x) -> -u(-x) of the equation, bit for bit (it exchanges
  the '+' and '-' split fluxes, so a wrong sign, mirror or index breaks it);
* constant states have a zero right-hand side.
"""
import numpy as np
import pytest

import oracle
from paper_2207_08500_amd import inputs
from tests._helpers import trained_params


def _grid(n, a=-1.0, b=1.0):
    dx = (b - a) / n
    return a + (np.arange(n) + 0.5) * dx, dx


@pytest.mark.parametrize("selector", [oracle.SEL_TENO, oracle.SEL_ALL_SMOOTH, oracle.SEL_MLP])
def test_conservation_periodic(selector):
    n = 150
    x, dx = _grid(n)
    u = 0.4 + np.sin(np.pi * x) + (np.abs(x) < 0.3) * 1.5
    P = trained_params() if selector == oracle.SEL_MLP else None
    u1, t, st = oracle.burgers_step(u, [0, n], dx, 0.3, 60, oracle.BC_PERIODIC, P, selector)
    assert st[0] == 0 and t[0] > 0
    assert abs(u1.sum() - u.sum()) <= 1e-12 * np.abs(u).sum()


def _characteristic_solution(x, t, u0):
    """Solve u = u0(x - u t) by Newton's method (valid before breaking)."""
    u = u0(x)
    for _ in range(60):
        xi = x - u * t
        g = u - u0(xi)
        h = 1e-7
        dg = 1 + t * (u0(xi + h) - u0(xi - h)) / (2 * h)
        u = u - g / dg
    return u


@pytest.mark.parametrize("selector", [oracle.SEL_ALL_SMOOTH, oracle.SEL_TENO])
def test_smooth_solution_order(selector):
    """u0 = 0.5 + 0.25 sin(pi x) on [-1, 1], periodic, t = 0.3 (waves break
    at t = 4/pi); the error falls at about fourth order."""
    u0 = lambda z: 0.5 + 0.25 * np.sin(np.pi * z)
    errs = []
    for n in (40, 80, 160):
        x, dx = _grid(n)
        cfl = 0.1
        # march to exactly t = 0.3 with the oracle's own CFL steps, then a last short step
        u, t, st = x * 0 + u0(x), np.zeros(1), np.zeros(1, np.int32)
        dt_max = cfl * dx / 0.75
        steps = int(np.ceil(0.3 / dt_max))
        # fixed dt = 0.3 / steps through the CFL number that gives it
        u, t, st = oracle.burgers_step(u, [0, n], dx, 0.0 + (0.3 / steps) * np.abs(u).max() / dx,
                                       1, oracle.BC_PERIODIC, None, selector)
        for _ in range(steps - 1):
            c = (0.3 / steps) * np.abs(u).max() / dx
            u, tt, st = oracle.burgers_step(u, [0, n], dx, c, 1, oracle.BC_PERIODIC, None, selector)
            t += tt
        assert abs(t[0] - 0.3) < 1e-12
        exact = _characteristic_solution(x, 0.3, u0)
        errs.append(np.abs(u - exact).mean())
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("Burgers smooth L1 errors %s, orders %s" % (errs, orders))
    assert min(orders) > 3.5


def test_shock_speed():
    n = 200
    x, dx = _grid(n, 0.0, 1.0)
    u = np.where(x < 0.2, 1.0, 0.0)
    t_end = 0.8
    u1, t, st = oracle.burgers_step(u, [0, n], dx, 0.4, int(np.ceil(t_end / (0.4 * dx))),
                                    oracle.BC_TRANSMISSIVE, None, oracle.SEL_TENO)
    # the CFL steps land near t_end; the shock sits at 0.2 + t / 2
    xs = 0.2 + 0.5 * t[0]
    i = np.argmax(u1 < 0.5)
    xc = x[i - 1] + (x[i] - x[i - 1]) * (u1[i - 1] - 0.5) / (u1[i - 1] - u1[i])
    assert abs(xc - xs) < 1.0 * dx, (xc, xs)
    assert u1.max() <= 1.0 + 1e-3 and u1.min() >= -1e-3  # no overshoot across the shock


def test_rarefaction_fan():
    n = 400
    x, dx = _grid(n, 0.0, 1.0)
    u = np.where(x < 0.3, 0.0, 1.0)
    u1, t, st = oracle.burgers_step(u, [0, n], dx, 0.4, int(0.4 / (0.4 * dx)),
                                    oracle.BC_TRANSMISSIVE, None, oracle.SEL_TENO)
    exact = np.clip((x - 0.3) / t[0], 0.0, 1.0)
    assert np.abs(u1 - exact).mean() < 4e-3


@pytest.mark.parametrize("selector", [oracle.SEL_TENO, oracle.SEL_MLP, oracle.SEL_ALL_SMOOTH])
@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_TRANSMISSIVE])
def test_mirror_symmetry_bitwise(selector, bc):
    n = 97
    rng = np.random.default_rng(5)
    u = rng.standard_normal(n) + np.where(np.arange(n) > 40, 2.0, -1.0)
    P = trained_params() if selector == oracle.SEL_MLP else None
    r, m, _ = oracle.burgers_rhs(u, [0, n], 0.01, bc, P, selector)
    rv, mv, _ = oracle.burgers_rhs(-u[::-1].copy(), [0, n], 0.01, bc, P, selector)
    assert np.array_equal(rv, -r[::-1])
    swapped = ((m[::-1] & 15) << 4) | (m[::-1] >> 4)
    assert np.array_equal(mv, swapped)


def test_constant_state_is_steady():
    for c in (0.0, 1.3, -2.0):
        r, m, st = oracle.burgers_rhs(np.full(50, c), [0, 50], 0.02, oracle.BC_PERIODIC, None,
                                      oracle.SEL_TENO)
        assert np.all(r == 0.0) and np.all(m == 0xFF)


def test_batched_lines_equal_single_lines():
    sizes = [7, 64, 130]
    u = np.concatenate([inputs.advection_c1(s, n) for s, n in zip((1, 2, 3), sizes)])
    off = np.concatenate([[0], np.cumsum(sizes)])
    dx = np.array([0.1, 0.03, 0.015])
    r, m, st = oracle.burgers_rhs(u, off, dx, oracle.BC_TRANSMISSIVE, None, oracle.SEL_TENO)
    for p in range(3):
        rp, mp, _ = oracle.burgers_rhs(u[off[p]:off[p + 1]], [0, sizes[p]], dx[p],
                                       oracle.BC_TRANSMISSIVE, None, oracle.SEL_TENO)
        assert np.array_equal(r[off[p]:off[p + 1]], rp)
        assert np.array_equal(m[off[p] + p:off[p + 1] + p + 1], mp)
