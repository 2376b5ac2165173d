"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point declared in include/neno6.h, and rejects bad arguments on
the host before touching a device."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "neno6.h")


def _lib():
    from paper_2207_08500_amd import native
    if not os.path.exists(native.LIB_PATH):
        from paper_2207_08500_amd import build
        build.build()
    return native, native.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(neno6_[a-z_0-9]+)\s*\(",
                                 text, re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("neno6_reconstruct", "neno6_rhs", "neno6_step", "neno6_classifier_train",
                 "neno6_mlp_prepare", "neno6_workspace_size", "neno6_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    native, lib = _lib()
    names = declared_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)
    assert set(native.EXPORTS) == set(names)


def test_host_argument_checks():
    native, lib = _lib()
    assert lib.neno6_version() >= 10000
    assert lib.neno6_status_string(-4).decode().startswith("state not physical")
    assert lib.neno6_mlp_prepared_bytes() >= 3228 * 4
    # invalid problems: workspace size 0, entry points return BAD_ARG before any launch
    ps = native.ProblemStruct()
    ps.equation = 7
    assert lib.neno6_workspace_size(C.byref(ps)) == 0
    ps.equation = native.EULER2D
    ps.nx, ps.ny, ps.dx2d, ps.dy2d, ps.gamma = 0, 4, 0.1, 0.1, 1.4
    assert lib.neno6_workspace_size(C.byref(ps)) == 0
    ps.nx = 8
    assert lib.neno6_workspace_size(C.byref(ps)) > 0
    assert lib.neno6_rhs(C.byref(ps), None, None, None, None, None, None, None, 0, None) == native.BAD_ARG
    # vector-Jacobian product: 2D scratch of 24 values per x and y face; the
    # advection right-hand side has its own adjoint entry point
    ps.precision = native.FP64
    nf2 = (8 + 1) * 4 + 8 * (4 + 1)
    assert lib.neno6_vjp_workspace_size(C.byref(ps)) >= 24 * nf2 * 8
    assert lib.neno6_rhs_vjp(C.byref(ps), None, None, None, None, None, 0, None) == native.BAD_ARG
    ps.precision = native.BF16
    assert lib.neno6_rhs_vjp(C.byref(ps), None, None, None, None, None, 0, None) == native.BAD_LAYOUT
    ps.precision = native.FP64
    # 1D: offsets must start at 0, increase strictly and end at total_cells
    import numpy as np
    off = np.array([0, 5, 5, 9], np.int64)
    p1 = native.ProblemStruct()
    p1.equation, p1.bc, p1.precision, p1.selector = native.EULER1D, 1, native.FP64, 1
    p1.n_problems, p1.total_cells, p1.gamma = 3, 9, 1.4
    p1.offsets = p1.dx = 1  # non-null device placeholders, never dereferenced on the host
    p1.offsets_host = off.ctypes.data
    assert lib.neno6_workspace_size(C.byref(p1)) == 0
    off[2] = 7
    assert lib.neno6_workspace_size(C.byref(p1)) > 0
    # launch shapes and flags are validated on the host
    p1.flags = 2
    assert lib.neno6_workspace_size(C.byref(p1)) == 0
    p1.flags = native.KEEP_MAP
    assert lib.neno6_workspace_size(C.byref(p1)) > 0
    for bad in ((3, 0, 0, 0), (4, -1, 0, 0), (4, 65537, 0, 0), (4, 0, 70000, 0), (4, 0, 0, 2)):
        tun = native.TuningStruct(*bad)
        p1.tuning = C.pointer(tun)
        assert lib.neno6_workspace_size(C.byref(p1)) == 0, bad
    tun = native.TuningStruct(8, 1024, 512, 1)
    p1.tuning = C.pointer(tun)
    assert lib.neno6_workspace_size(C.byref(p1)) > 0
    # the autotuner takes reduced-precision Euler problems with the classifier only
    best = native.TuningStruct()
    assert lib.neno6_autotune(C.byref(p1), None, None, None, 0, 3, C.byref(best), None,
                              None) == native.UNSUPPORTED
    p1.precision, p1.selector = native.BF16, native.SEL_MLP
    assert lib.neno6_autotune(C.byref(p1), None, None, None, 0, 3, C.byref(best), None,
                              None) == native.BAD_ARG
    # lines beyond 32-bit re-check queue entries are refused
    big = np.array([0, 1 << 29], np.int64)
    p2 = native.ProblemStruct()
    p2.equation, p2.bc, p2.precision, p2.selector = native.EULER1D, 1, native.BF16, 1
    p2.n_problems, p2.total_cells, p2.gamma = 1, 1 << 29, 1.4
    p2.offsets = p2.dx = 1
    p2.offsets_host = big.ctypes.data
    assert lib.neno6_workspace_size(C.byref(p2)) == 0
    assert lib.neno6_reconstruct(None, None, 10, 2, 0, 1, None, None, None, None) == native.BAD_ARG
    # batches of 2D grids: workspace of the largest grid, every grid checked,
    # no re-check counters and no allocation-free entry point for batches
    g3 = [(67, 45, 1 / 67, 1 / 45), (130, 3, 1 / 130, 1 / 3), (64, 64, 1 / 64, 1 / 64)]
    pb = native.Problem(native.EULER2D, native.FP16, grids=g3, device="cpu")
    sizes = [native.Problem(native.EULER2D, native.FP16, nx=a, ny=b_, dx2d=c, dy2d=d,
                            device="cpu") for a, b_, c, d in g3]
    assert lib.neno6_workspace_size(C.byref(pb.struct())) == max(
        lib.neno6_workspace_size(C.byref(x.struct())) for x in sizes)
    assert pb.n_faces == sum(x.n_faces for x in sizes) and pb.total_cells == 67 * 45 + 130 * 3 + 64 * 64
    bad = native.Problem(native.EULER2D, native.FP16, grids=g3 + [(0, 5, 0.1, 0.1)], device="cpu")
    assert lib.neno6_workspace_size(C.byref(bad.struct())) == 0
    cnt = (C.c_uint32 * 2)()
    assert lib.neno6_recheck_count(C.byref(pb.struct()), None, None, 0, cnt, None) == native.UNSUPPORTED
    assert lib.neno6_rhs_noalloc(C.byref(pb.struct()), None, None, None, None, None, None,
                                 None) == native.UNSUPPORTED
    # re-check arithmetic: FP32 or two-part FP16 only (placeholders, never dereferenced)
    bad_mode = native.MlpStruct(1, 1, 0.5, 2)
    assert lib.neno6_mlp_logits(C.byref(bad_mode), native.FP16, C.c_void_p(1), 10, C.c_void_p(1), None,
                                None) == native.BAD_ARG
    assert lib.neno6_reconstruct(None, None, 10, 1, 0, 0, None, None, None, None) == native.BAD_ARG
    assert lib.neno6_classifier_train(None, None, None, None, None, None, None, 0, 0, 0.0, 0.9,
                                      0.999, 1e-8, native.BF16, None, None, 0, None) == native.BAD_ARG


def test_product_path_does_not_import_the_oracle():
    """The HIP binding never reaches the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2207_08500_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "neno6_oracle" not in text, f
