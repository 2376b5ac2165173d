"""Labelled training data after the paper's data pipeline (Sec. 3.2, Alg. 1
and the function families of the appendix table "Parameters for training and
validation datasets generation").

For each grid N in {50, 100, 200} (40 / 40 / 20 % of the samples) a function
of one of the nine families is drawn on [-1, 1] (cell-centred values), either
as it is ("analytic") or evolved in time by the linear advection or the
Burgers equation ("evolved"); six-point stencils are cut at interior cell
interfaces x_{i+1/2} and every candidate S_k gets the flag eta_k (1: the
candidate holds a genuine discontinuity and must be dropped).

Labels:
* analytic families whose singular points are known in closed form (4
  triangle kinks, 5 the kink at x0, 7 the edges of the ellipse, 8 the step;
  1-3 are smooth): eta_k = 1 iff a singular point lies strictly inside the
  cells of S_k;
* families 6 and 9 (flag "0/1" without a closed-form singular point) and all
  evolved solutions: the TENO6-opt selection (NENO6_SEL_TENO), eta = 1 - delta.

Evolution and TENO labelling run on the GPU through the library (batched
lines, FP64); the families are sampled on the host.  Output: raw stencils
s[n][6] (FP64; the trainer applies eq. normalizainput) and labels y[n]
(bit k = eta_k), in the layout neno6_classifier_train takes.

Readings (not fixed by the text): a_k ~ U[0.1, 2] (family 2); family 6 is
the printed polynomial sum with integer k_i; family 8's x0 is drawn on the
grid's interfaces in [-0.6, 0.6] (the data point is the interface at x0);
family 9 uses N_f = N / 4 (wavelength four cells); evolved samples: half
advection to t ~ U[0, 1], half Burgers to t ~ U[0, 0.5], periodic, CFL 0.4;
half of the samples are analytic, half evolved; at most 8 interfaces per
function (family 8: one).
"""
from __future__ import annotations

import numpy as np
import torch

from . import native

from .inputs import ALG1_GRIDS as GRIDS, ALG1_GRID_SHARE as GRID_SHARE  # noqa: E402
from .inputs import alg1_family as _family, alg1_geometric_labels as geometric_labels  # noqa: E402


def _teno_labels(u_lines, N, dev):
    """TENO6-opt masks of every face of periodic lines u_lines[m][N] (one call)."""
    m = u_lines.shape[0]
    off = np.arange(m + 1, dtype=np.int64) * N
    prob = native.Problem(native.ADVECTION, native.FP64, native.SEL_TENO, native.PERIODIC, off,
                          np.full(m, 2.0 / N), device=dev)
    u = torch.as_tensor(u_lines.reshape(-1), dtype=torch.float64, device=dev).contiguous()
    masks = torch.zeros(prob.mask_count(), dtype=torch.uint8, device=dev)
    native.neno6_rhs(prob, None, u, torch.zeros_like(u), prob.workspace(dev), masks_out=masks)
    torch.cuda.synchronize(dev)
    # face k of line p is global face p * (N + 1) + k (face k between cells k-1 and k)
    return masks.cpu().numpy().reshape(m, N + 1) & 15


def _evolve(u_lines, N, equation, t_end, dev):
    m = u_lines.shape[0]
    off = np.arange(m + 1, dtype=np.int64) * N
    prob = native.Problem(equation, native.FP64, native.SEL_TENO, native.PERIODIC, off,
                          np.full(m, 2.0 / N), device=dev)
    u = torch.as_tensor(u_lines.reshape(-1), dtype=torch.float64, device=dev).contiguous()
    t = torch.zeros(m, dtype=torch.float64, device=dev)
    st = torch.zeros(m, dtype=torch.int32, device=dev)
    ws = prob.workspace(dev)
    # march every line with the same number of CFL steps, enough for the
    # largest requested time; lines keep their own dt (their own max |u|)
    dx = 2.0 / N
    speed = np.maximum(np.abs(u_lines).max(axis=1), 1e-12) if equation == native.BURGERS else np.ones(m)
    n_steps = int(np.ceil((t_end * speed / (0.4 * dx)).max())) if t_end > 0 else 0
    if n_steps:
        native.neno6_step(prob, None, u, 0.4, min(n_steps, 4000), t, st, ws)
    torch.cuda.synchronize(dev)
    ok = st.cpu().numpy() == 0
    return u.cpu().numpy().reshape(m, N), ok


def generate(n_samples: int, seed: int, device="cuda", per_function: int = 8):
    """Returns (s[n][6] FP64 raw stencils, y[n] uint8 labels, kind[n] uint8)
    with kind 0 = analytic with closed-form labels, 1 = analytic labelled by
    TENO6-opt, 2 = evolved (TENO6-opt labels)."""
    native.load()
    dev = torch.device(device)
    g = np.random.Generator(np.random.PCG64([seed, 2207085000, 9]))
    S, Y, K = [], [], []
    n_done = 0
    while n_done < n_samples:
        N = int(g.choice(GRIDS, p=GRID_SHARE))
        dx = 2.0 / N
        x = -1.0 + (np.arange(N) + 0.5) * dx
        batch = 64
        fams = g.integers(1, 10, batch)
        funcs = [_family(g, int(f), N) for f in fams]
        U = np.stack([f(x) for f, _ in funcs]).astype(np.float64)
        evolved = g.random() < 0.5
        if evolved:
            eq = native.ADVECTION if g.random() < 0.5 else native.BURGERS
            t_end = g.uniform(0, 1.0) if eq == native.ADVECTION else g.uniform(0, 0.5)
            U, ok = _evolve(U, N, eq, t_end, dev)
            labels_all = _teno_labels(U, N, dev)
        else:
            ok = np.ones(batch, bool)
            labels_all = None
            if any(sing is None for _, sing in funcs):
                labels_all = _teno_labels(U, N, dev)
        for m in range(batch):
            if not ok[m] or not np.all(np.isfinite(U[m])):
                continue
            fam, (_, sing) = int(fams[m]), funcs[m]
            if fam == 8 and not evolved:
                faces = [int(round((sing[0] + 1.0) / dx)) - 1]  # face x_{i+1/2} = x0
            else:
                faces = g.choice(np.arange(3, N - 4), size=min(per_function, N - 7), replace=False)
            sten = np.stack([U[m, i - 2:i + 4] for i in faces])
            if evolved or sing is None:
                # TENO mask of face x_{i+1/2} is at face index i + 1 of the line
                y = (~labels_all[m, np.asarray(faces) + 1]) & 15
                kind = 2 if evolved else 1
            else:
                y = geometric_labels(faces, sing, N)
                kind = 0
            S.append(sten)
            Y.append(y.astype(np.uint8))
            K.append(np.full(len(faces), kind, np.uint8))
            n_done += len(faces)
            if n_done >= n_samples:
                break
    return (np.concatenate(S)[:n_samples], np.concatenate(Y)[:n_samples],
            np.concatenate(K)[:n_samples])
