"""Seeded synthetic inputs for the NENO6 workloads.

This module only draws random numbers and lays out initial data; it holds none
of the reconstruction's arithmetic.  Both the HIP library's tests/benchmark and
the CPU oracle take their inputs from here, so the two sides see identical
data.  Every generator takes an integer seed and uses numpy's PCG64.

Workloads (shapes follow the paper's test cases: 1D grids of a few hundred
cells, 2D Riemann problems of the four-quadrant type, Sec. 4):
  * ``advection_c1``    -- periodic 1D advection data on [-1, 1]
  * ``riemann1d_batch`` -- batches of 1D Euler Riemann problems (shock tubes)
  * ``riemann2d``       -- a 2D four-quadrant Riemann problem with a density wave
  * ``uneven_sizes``    -- log-uniform line lengths for batched runs
  * ``classifier_samples`` -- six-point stencils with per-candidate labels
  * ``alg1_family``     -- the function families of the paper's training-set
                           construction (Alg. 1 and its parameter table)
  * ``mlp_init``        -- a seeded parameter block for the 6-64-32-16-8-4 network
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 2207085000
GAMMA = 1.4
WIDTHS = (6, 64, 32, 16, 8, 4)
NPARAM = sum(WIDTHS[i] * WIDTHS[i + 1] + WIDTHS[i + 1] for i in range(5))  # 3228

# Stencil span of each candidate in six-point positions 0..5 (cells i-2..i+3):
# S0 = {i-1,i,i+1}, S1 = {i,i+1,i+2}, S2 = {i-2,i-1,i}, S3 = {i,...,i+3}.
CANDIDATE_SPAN = ((1, 3), (2, 4), (0, 2), (2, 5))


def rng(seed: int, *stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), *[int(s) for s in stream]]))


# --------------------------------------------------------------------------
# Classifier parameters
# --------------------------------------------------------------------------
def mlp_init(seed: int = BASE_SEED) -> np.ndarray:
    """He-uniform weights, small uniform biases; packed FP64 block
    W1[64][6] b1 W2[32][64] b2 W3[16][32] b3 W4[8][16] b4 W5[4][8] b5."""
    g = rng(seed, 11)
    parts = []
    for i in range(5):
        nin, nout = WIDTHS[i], WIDTHS[i + 1]
        lim = np.sqrt(6.0 / nin)
        parts.append(g.uniform(-lim, lim, size=nout * nin))
        parts.append(g.uniform(-0.1, 0.1, size=nout))
    p = np.concatenate(parts)
    assert p.size == NPARAM
    return p


def split_params(p: np.ndarray):
    """Views (W_l [out][in], b_l [out]) for l = 1..5."""
    out, o = [], 0
    for i in range(5):
        nin, nout = WIDTHS[i], WIDTHS[i + 1]
        W = p[o:o + nout * nin].reshape(nout, nin)
        o += nout * nin
        b = p[o:o + nout]
        o += nout
        out.append((W, b))
    return out


# --------------------------------------------------------------------------
# 1D scalar advection on [-1, 1], periodic, cell-centred
# --------------------------------------------------------------------------
def cell_centres(n: int, a: float, b: float) -> np.ndarray:
    dx = (b - a) / n
    return a + (np.arange(n) + 0.5) * dx


def advection_c1(seed: int = BASE_SEED, n: int = 200) -> np.ndarray:
    """Two sines (integer wavenumber 1-4 so the data is 2-periodic, amplitude
    0.1-1), two square pulses and one triangle at random positions."""
    g = rng(seed, 1)
    x = cell_centres(n, -1.0, 1.0)
    u = np.zeros(n)
    for _ in range(2):
        k = g.integers(1, 5)
        A = g.uniform(0.1, 1.0)
        phi = g.uniform(0.0, 2 * np.pi)
        u += A * np.sin(np.pi * k * x + phi)

    def wrapped_dist(xc):
        d = x - xc
        return d - 2.0 * np.round(d / 2.0)

    for _ in range(2):
        h = g.uniform(0.1, 1.0)
        w = g.uniform(0.1, 0.4)
        xc = g.uniform(-1.0, 1.0)
        u += np.where(np.abs(wrapped_dist(xc)) < 0.5 * w, h, 0.0)
    h = g.uniform(0.1, 1.0)
    hw = g.uniform(0.05, 0.2)
    xc = g.uniform(-1.0, 1.0)
    u += h * np.maximum(0.0, 1.0 - np.abs(wrapped_dist(xc)) / hw)
    return u


# --------------------------------------------------------------------------
# Euler initial data
# --------------------------------------------------------------------------
def _state_draw(g, size):
    rho = g.uniform(0.1, 1.0, size)
    u = g.uniform(-1.0, 1.0, size)
    p = np.exp(g.uniform(np.log(0.1), np.log(1000.0), size))
    return rho, u, p


def conservative1d(rho, u, p, gamma=GAMMA):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def conservative2d(rho, u, v, p, gamma=GAMMA):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def riemann1d_batch(seed: int = BASE_SEED, sizes=(4000,) * 256, perturb=False,
                    gamma: float = GAMMA):
    """Concatenated 1D Riemann problems on [0, 1].

    Left/right states: rho ~ U[0.1, 1], u ~ U[-1, 1], p ~ log-uniform[0.1, 1000];
    diaphragm at x0 ~ U[0.2, 0.8].  With ``perturb`` the density also carries
    a sinusoidal wave (amplitude 0.2, wavenumber 1-8), multiplicative; with
    ``perturb="odd"`` only the problems of odd index do (the others are
    those of the unperturbed batch).
    Returns (q [3][total] FP64, offsets [n+1] int64, dx [n] FP64)."""
    if perturb not in (False, True, "odd"):
        raise ValueError("perturb: False, True or 'odd'")
    sizes = np.asarray(sizes, dtype=np.int64)
    g = rng(seed, 2, int(sizes.size))
    offsets = np.zeros(sizes.size + 1, np.int64)
    offsets[1:] = np.cumsum(sizes)
    q = np.zeros((3, int(offsets[-1])))
    dx = 1.0 / sizes.astype(np.float64)
    rl, ul, pl = _state_draw(g, sizes.size)
    rr, ur, pr = _state_draw(g, sizes.size)
    x0 = g.uniform(0.2, 0.8, sizes.size)
    kw = g.integers(1, 9, sizes.size)
    for i, n in enumerate(sizes):
        x = cell_centres(int(n), 0.0, 1.0)
        left = x < x0[i]
        rho = np.where(left, rl[i], rr[i])
        if perturb is True or (perturb == "odd" and i % 2 == 1):
            rho = rho * (1.0 + 0.2 * np.sin(2 * np.pi * kw[i] * x))
        u = np.where(left, ul[i], ur[i])
        p = np.where(left, pl[i], pr[i])
        q[:, offsets[i]:offsets[i + 1]] = conservative1d(rho, u, p, gamma)
    return q, offsets, dx


def uneven_sizes(seed: int = BASE_SEED, n_problems: int = 4096, lo: int = 256, hi: int = 16384):
    g = rng(seed, 4)
    return np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), n_problems))).astype(np.int64)


def riemann2d(seed: int = BASE_SEED, nx: int = 2048, ny: int = 2048, gamma: float = GAMMA):
    """Four-quadrant Riemann data on [0,1]^2 split at (0.5, 0.5); per-quadrant
    (rho, u, v, p) drawn as for 1D; rho multiplied by 1 + 0.2 sin(2 pi (kx x + ky y))
    with kx, ky ~ U{1..8}.  Returns q [4][ny][nx] FP64."""
    g = rng(seed, 3)
    rho_q = g.uniform(0.1, 1.0, 4)
    u_q = g.uniform(-1.0, 1.0, 4)
    v_q = g.uniform(-1.0, 1.0, 4)
    p_q = np.exp(g.uniform(np.log(0.1), np.log(1000.0), 4))
    kx, ky = g.integers(1, 9, 2)
    x = cell_centres(nx, 0.0, 1.0)[None, :]
    y = cell_centres(ny, 0.0, 1.0)[:, None]
    quad = (x >= 0.5).astype(np.int64) + 2 * (y >= 0.5).astype(np.int64)
    rho = rho_q[quad] * (1.0 + 0.2 * np.sin(2 * np.pi * (kx * x + ky * y)))
    return conservative2d(rho, u_q[quad], v_q[quad], p_q[quad], gamma)


# --------------------------------------------------------------------------
# Classifier training samples
# --------------------------------------------------------------------------
def classifier_samples(seed: int = BASE_SEED, n: int = 1 << 16):
    """Six-point stencils f(x_c + j dx), j = -2..3, with the label of each
    candidate sub-stencil (bit k set = candidate k crossed by a discontinuity).

    dx = 2/N with N in {50, 100, 200} at 40/40/20 %, x_c ~ U[-1, 1].
    Half smooth: polynomials of degree 0-5 (coefficients U[-1,1] in x - x_c) or
    A sin(w x + phi), w ~ U[0.5, 20], A ~ log-uniform[1e-2, 1e2]; all labels 0.
    Half discontinuous at x_d ~ U(x_{-2}, x_3): a step (a | a r) or a kink
    (slopes s, s r), a, s = +-U[0.1, 1], r ~ log-uniform[1e-3, 1e3]; candidate k
    is labelled 1 iff x_d lies strictly inside its span.
    Returns (s [n][6] FP64, y [n] uint8)."""
    g = rng(seed, 5, n)
    N = g.choice(np.array([50, 100, 200]), size=n, p=[0.4, 0.4, 0.2])
    dx = 2.0 / N
    xc = g.uniform(-1.0, 1.0, n)
    j = np.arange(-2, 4)[None, :]
    xs = xc[:, None] + j * dx[:, None]
    s = np.zeros((n, 6))
    y = np.zeros(n, np.uint8)
    smooth = np.arange(n) < n // 2
    g.shuffle(smooth)
    kind = g.integers(0, 2, n)  # smooth: 0 poly 1 sine; disc: 0 step 1 kink
    # smooth: polynomials
    deg = g.integers(0, 6, n)
    coef = g.uniform(-1.0, 1.0, (n, 6))
    coef = np.where(np.arange(6)[None, :] <= deg[:, None], coef, 0.0)
    t = xs - xc[:, None]
    poly = np.zeros((n, 6))
    for d in range(5, -1, -1):
        poly = poly * t + coef[:, d:d + 1]
    w = g.uniform(0.5, 20.0, n)
    phi = g.uniform(0.0, 2 * np.pi, n)
    A = np.exp(g.uniform(np.log(1e-2), np.log(1e2), n))
    sine = A[:, None] * np.sin(w[:, None] * xs + phi[:, None])
    # discontinuous
    xd = g.uniform(xs[:, 0], xs[:, 5])
    a = g.uniform(0.1, 1.0, n) * g.choice(np.array([-1.0, 1.0]), n)
    r = np.exp(g.uniform(np.log(1e-3), np.log(1e3), n))
    right = xs > xd[:, None]
    step = np.where(right, (a * r)[:, None], a[:, None])
    dxd = xs - xd[:, None]
    kink = np.where(right, (a * r)[:, None] * dxd, a[:, None] * dxd)
    s = np.where(smooth[:, None], np.where((kind == 0)[:, None], poly, sine),
                 np.where((kind == 0)[:, None], step, kink))
    for k, (lo, hi) in enumerate(CANDIDATE_SPAN):
        inside = (xd > xs[:, lo]) & (xd < xs[:, hi])
        y |= np.where(~smooth & inside, np.uint8(1 << k), np.uint8(0)).astype(np.uint8)
    return np.ascontiguousarray(s), y


# --------------------------------------------------------------------------
# Counter-based classifier samples: the same distribution as
# classifier_samples, drawn per sample from Philox4x32-10 (Salmon, Moraes,
# Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011) so
# that any range of samples can be generated on the device independently.
# This is the host twin of the library's generator: sample i uses the
# counters (lo(i), hi(i), b, 0x43355331) for b = 0..4 and the key (lo(seed),
# hi(seed)); a 32-bit word w gives the uniform (w + 1/2) 2^-32; every value is
# formed in FP64 with separately rounded operations in the order written
# here, then rounded to FP32.
# --------------------------------------------------------------------------
PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)
C5_STREAM = 0x43355331
LN_1EM2, LN_1E2 = float.fromhex("-0x1.26bb1bbb55515p+2"), float.fromhex("0x1.26bb1bbb55516p+2")
LN_1EM3, LN_1E3 = float.fromhex("-0x1.ba18a998fffa0p+2"), float.fromhex("0x1.ba18a998fffa0p+2")
TWO_PI = float.fromhex("0x1.921fb54442d18p+2")


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32 with 10 rounds: ctr [..., 4] uint32, key (k0, k1)."""
    c = [np.asarray(ctr[..., i], np.uint32) for i in range(4)]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W[0]) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W[1]) & 0xFFFFFFFF
        p0 = np.uint64(PHILOX_M[0]) * c[0].astype(np.uint64)
        p1 = np.uint64(PHILOX_M[1]) * c[2].astype(np.uint64)
        c = [(p1 >> np.uint64(32)).astype(np.uint32) ^ c[1] ^ np.uint32(k0), p1.astype(np.uint32),
             (p0 >> np.uint64(32)).astype(np.uint32) ^ c[3] ^ np.uint32(k1), p0.astype(np.uint32)]
    return np.stack(c, axis=-1)


def classifier_samples_philox(seed: int = BASE_SEED, first: int = 0, n: int = 1 << 16):
    """Samples first .. first+n-1 of the counter-based generator.

    Per sample: N in {50, 100, 200} at 40/40/20 %, dx = 2/N, x_c ~ U[-1, 1],
    cells x_j = x_c + (j - 2) dx, j = 0..5; smooth with probability 1/2, then
    a polynomial of degree 0-5 in t = (j - 2) dx (coefficients U[-1, 1],
    Horner) or A sin(w x + phi) (w ~ U[0.5, 20], phi ~ U[0, 2 pi], A
    log-uniform in [1e-2, 1e2]), labels 0; else a jump at x_d ~ U(x_0, x_5): a
    step (a | a r) or a kink ((x - x_d) a | (x - x_d) a r), a = +-U[0.1, 1],
    r log-uniform in [1e-3, 1e3], and candidate k labelled 1 iff x_d lies
    strictly inside its span (FP64 comparisons).
    Returns (s [n][6] FP32, y [n] uint8, s64 [n][6] FP64 before rounding)."""
    i = np.arange(first, first + n, dtype=np.uint64)
    ctr = np.zeros((5, n, 4), np.uint32)
    ctr[:, :, 0] = (i & np.uint64(0xFFFFFFFF)).astype(np.uint32)[None, :]
    ctr[:, :, 1] = (i >> np.uint64(32)).astype(np.uint32)[None, :]
    ctr[:, :, 2] = np.arange(5, dtype=np.uint32)[:, None]
    ctr[:, :, 3] = C5_STREAM
    words = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))  # [5][n][4]
    u = (words.astype(np.float64) + 0.5) * 2.0 ** -32
    N = np.where(u[0, :, 0] < 0.4, 50.0, np.where(u[0, :, 0] < 0.8, 100.0, 200.0))
    dx = 2.0 / N
    xc = -1.0 + 2.0 * u[0, :, 1]
    smooth = u[0, :, 2] < 0.5
    kind = u[0, :, 3] >= 0.5
    t = np.arange(-2, 4, dtype=np.float64)[None, :] * dx[:, None]
    xs = xc[:, None] + t
    deg = np.minimum(np.floor(6.0 * u[1, :, 0]), 5.0)
    coef = np.stack([u[2, :, 0], u[2, :, 1], u[2, :, 2], u[2, :, 3], u[3, :, 0], u[3, :, 1]], axis=1)
    coef = np.where(np.arange(6)[None, :] <= deg[:, None], -1.0 + 2.0 * coef, 0.0)
    poly = np.zeros((n, 6))
    for d in range(5, -1, -1):
        poly = poly * t + coef[:, d:d + 1]
    w = 0.5 + 19.5 * u[1, :, 1]
    phi = TWO_PI * u[1, :, 2]
    A = np.exp(LN_1EM2 + u[1, :, 3] * (LN_1E2 - LN_1EM2))
    sine = A[:, None] * np.sin(w[:, None] * xs + phi[:, None])
    xd = xs[:, 0] + u[3, :, 2] * (xs[:, 5] - xs[:, 0])
    a = (0.1 + 0.9 * u[3, :, 3]) * np.where(u[4, :, 0] < 0.5, -1.0, 1.0)
    r = np.exp(LN_1EM3 + u[4, :, 1] * (LN_1E3 - LN_1EM3))
    right = xs > xd[:, None]
    amp = np.where(right, (a * r)[:, None], a[:, None])
    disc = np.where(kind[:, None], amp * (xs - xd[:, None]), amp)
    s64 = np.where(smooth[:, None], np.where(kind[:, None], sine, poly), disc)
    y = np.zeros(n, np.uint8)
    for k, (lo, hi) in enumerate(CANDIDATE_SPAN):
        inside = (xd > xs[:, lo]) & (xd < xs[:, hi])
        y |= np.where(~smooth & inside, np.uint8(1 << k), np.uint8(0)).astype(np.uint8)
    return np.ascontiguousarray(s64.astype(np.float32)), y, np.ascontiguousarray(s64)


def epoch_permutation(seed: int, epoch: int, n: int) -> np.ndarray:
    """The sample order of one training epoch (reshuffled every epoch)."""
    return rng(seed, 6, epoch).permutation(n).astype(np.int64)


# --------------------------------------------------------------------------
# Generic helpers for tests
# --------------------------------------------------------------------------
def random_stencils(seed: int, n: int, scale: float = 1.0) -> np.ndarray:
    """Stencils mixing smooth, jump and noisy data at several magnitudes."""
    g = rng(seed, 7, n)
    base = g.standard_normal((n, 6))
    mag = np.exp(g.uniform(np.log(1e-3), np.log(1e3), n))[:, None]
    return np.ascontiguousarray(scale * base * mag)


# --------------------------------------------------------------------------
# Function families of the training-set construction (Alg. 1 and the
# appendix table of parameters for training and validation data): a
# function of family 1..9 drawn on [-1, 1] with its singular points (None
# where the family has none in closed form).  Readings: a_k ~ U[0.1, 2]
# (family 2); family 6 with integer exponents; family 8's x0 on a grid
# interface in [-0.6, 0.6]; family 9 with N_f = N / 4.
# --------------------------------------------------------------------------
ALG1_GRIDS = (50, 100, 200)
ALG1_GRID_SHARE = (0.4, 0.4, 0.2)
# candidate cell offsets relative to cell i (face x_{i+1/2} between i, i+1)
ALG1_CAND_CELLS = ((-1, 0, 1), (0, 1, 2), (-2, -1, 0), (0, 1, 2, 3))


def alg1_family(g, fam, N):
    """Returns (f(x) vectorised, list of singular points or None for TENO labels)."""
    dx = 2.0 / N
    if fam == 1:
        k = g.uniform(-5, 5)
        return (lambda x: k * x), []
    if fam == 2:
        k, a = g.uniform(1, 5), g.uniform(0.1, 2.0)
        return (lambda x: a * np.sin(k * x)), []
    if fam == 3:
        a1, a2 = g.uniform(-1, 1, 2)
        return (lambda x: np.exp(a1 * (x - a2) ** 2)), []
    if fam == 4:
        r, P = g.uniform(1, 3), g.uniform(2 * dx, 8 * dx)
        f = lambda x: (r / P) * (P - np.abs(np.mod(x, 2 * P) - P))
        kinks = [m * P for m in range(int(np.floor(-1.2 / P)), int(np.ceil(1.2 / P)) + 1)]
        return f, kinks
    if fam == 5:
        b1, x0, c = g.normal(0.0, np.sqrt(0.6)), g.uniform(-0.6, 0.6), g.uniform(0, 1)
        return (lambda x: np.maximum(0.0, b1 * (x - x0)) + c), [x0]
    if fam == 6:
        k1, k2 = g.integers(2, 9, 2)
        a1, a2 = g.uniform(0, 2, 2)
        return (lambda x: (x - a1) ** k1 + (x - a2) ** k2), None
    if fam == 7:
        al, a = g.uniform(0, 2, 2)
        al = max(al, 1e-3)
        f = lambda x: np.sqrt(np.maximum(0.0, 1.0 - al * al * (x - a) ** 2))
        return f, [a - 1.0 / al, a + 1.0 / al]
    if fam == 8:
        xl, xr = g.uniform(0, 2, 2)
        i0 = int(g.integers(int(0.2 * N), int(0.8 * N)))
        x0 = -1.0 + i0 * dx  # an interface
        return (lambda x: np.where(x <= x0, xl, xr)), [x0]
    a1, x0 = g.uniform(0, 2, 2)
    Nf = N / 4
    return (lambda x: a1 * np.sin(Nf * np.pi * (x - x0))), None


def alg1_geometric_labels(faces, singular, N):
    """eta[k] per face index i (face x_{i+1/2}) from singular points."""
    dx = 2.0 / N
    y = np.zeros(len(faces), np.uint8)
    sp = np.asarray(singular, np.float64)
    for n, i in enumerate(faces):
        for k, cells in enumerate(ALG1_CAND_CELLS):
            lo = -1.0 + (i + cells[0]) * dx  # left edge of the first cell
            hi = -1.0 + (i + cells[-1] + 1) * dx  # right edge of the last cell
            if np.any((sp > lo) & (sp < hi)):
                y[n] |= 1 << k
    return y
