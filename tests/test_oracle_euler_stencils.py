"""The oracle's export of the 1D Euler classifier inputs (euler1d_stencils,
used to build classifier training data) against its right-hand side: the
TENO6-opt labels of the exported stencils are the masks the right-hand side
reports, and the exported stencils, combined with every candidate kept and
projected back with the Roe eigenvectors, give the right-hand side's face
fluxes (Sec. 4.4: characteristic Rusanov split)."""
import numpy as np
import pytest

import oracle
from paper_2207_08500_amd import inputs


@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_TRANSMISSIVE])
def test_stencils_reproduce_the_rhs(bc):
    sizes = (30, 41)
    q, off, dx = inputs.riemann1d_batch(12, sizes)
    S = oracle.euler1d_stencils(q, off, 1.4, bc)
    nf = int(off[-1]) + len(sizes)
    assert S.shape == (nf, 6, 6)
    # TENO6-opt labels of the exported stencils = the masks of the rhs
    _, m, _ = oracle.euler1d_rhs(q, off, dx, 1.4, bc, None, oracle.SEL_TENO)
    kept = oracle.teno(S.reshape(-1, 6))[3].astype(np.uint8).reshape(nf, 3, 2)
    assert np.array_equal(kept[:, :, 0] | (kept[:, :, 1] << 4), m.T)
    # all candidates kept: h = sum_j a_j s_j with the linear weights' coefficients
    a = oracle.linear_weights() @ oracle.candidate_coeffs()
    r, _, _ = oracle.euler1d_rhs(q, off, dx, 1.4, bc, None, oracle.SEL_ALL_SMOOTH)
    for p in range(len(sizes)):
        o, n = int(off[p]), sizes[p]
        F = np.zeros((n + 1, 3))
        for k in range(n + 1):
            f = o + p + k
            cl = (k - 1) % n if bc == oracle.BC_PERIODIC else min(max(k - 1, 0), n - 1)
            cr = k % n if bc == oracle.BC_PERIODIC else min(k, n - 1)
            _, R = oracle.euler1d_eigen(q[:, o + cl], q[:, o + cr], 1.4)
            hs = np.array([a @ S[f, 2 * mm] + a @ S[f, 2 * mm + 1] for mm in range(3)])
            F[k] = R @ hs
        want = r[:, o:o + n].T
        got = (F[:-1] - F[1:]) / dx[p]
        assert np.allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
