"""Launches the hot kernels on the benchmark workloads for profiling, plus a
plain device copy of known size that calibrates the memory counters.

    rocprofv3 --pmc FETCH_SIZE --kernel-trace --output-format csv -d OUT -o run -- \
        python3 paper_2207_08500_amd/profile_kernels.py --tuned --no-fp64
    rocprofv3 --pmc WRITE_SIZE --kernel-trace --output-format csv -d OUT -o run -- \
        python3 paper_2207_08500_amd/profile_kernels.py --tuned --no-fp64
    rocprofv3 --kernel-trace --stats --output-format csv -d OUT -o run -- \
        python3 paper_2207_08500_amd/profile_kernels.py --steps 20

Workloads (--workload): c4, 4096 independent 1D Euler Riemann problems with N
log-uniform in [256, 16384] (default); c2, 256 problems of 4000 cells.  FP32
state, FP16/BF16 classifier.  Without --steps: the right-hand-side pass as it
runs inside a step (the fused face kernel with the re-check at the
stated margins and the flux difference, face map kept) --reps times in FP16
and in BF16, the FP64 plain path once, then the copy.  With --tuned the
launches take the shape the autotuner picks for the FP16 pass (as the benchmark does;
it prints the shape); with --shape W,B that many waves per workgroup and
workgroups; else the library default.  With --steps K: instead, K SSP-RK3
steps of the FP16 path with the re-check, captured once in a HIP graph and
replayed after about 0.1 s of warm-up replays, in the --shape launch shape if
given, else the autotuner's; a one-element torch fill right before the timed
replays marks where they start in a kernel trace.  --2d: the 2D Euler
four-quadrant Riemann problem on 2048 x 2048 cells instead of a 1D batch.
--perturb-odd: the 1D batch with the density wave in every problem of odd
index (smooth regions where the plain batch has constant states).
"""
import argparse
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2207_08500_amd import inputs, native  # noqa: E402

def _margins():
    """The stated re-check margins of the committed weights."""
    import json
    with open(os.path.join(ROOT, "tests", "golden", "neno6_mlp_trained_margins.json")) as f:
        m = json.load(f)["margin"]
    return {native.BF16: float(m["bf16"]), native.FP16: float(m["fp16"])}


MARGIN = _margins()


def batch(workload, perturb=False):
    if workload == "c4":
        sizes = inputs.uneven_sizes(inputs.BASE_SEED, 4096, 256, 16384)
    else:
        sizes = np.full(256, 4000, np.int64)
    return inputs.riemann1d_batch(inputs.BASE_SEED, sizes, perturb=perturb)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--steps", type=int, default=0)
    ap.add_argument("--tuned", action="store_true")
    ap.add_argument("--shape", default=None, help="W,B: waves per workgroup, workgroups")
    ap.add_argument("--workload", choices=("c4", "c2"), default="c4")
    ap.add_argument("--2d", dest="two_d", action="store_true")
    ap.add_argument("--perturb-odd", action="store_true",
                    help="every problem of odd index with the density wave (no constant states)")
    a = ap.parse_args()
    native.load()
    dev = torch.device("cuda:0")
    P = np.load(os.path.join(ROOT, "tests", "golden", "neno6_mlp_trained.npy"), allow_pickle=False)
    if a.steps > 0 and a.two_d:
        return step_replay_2d(a.steps, P, dev)
    q0, off, dx = batch(a.workload, "odd" if a.perturb_odd else False)
    q32 = torch.as_tensor(q0, dtype=torch.float32, device=dev).contiguous()
    if a.steps > 0:
        return step_replay(a.steps, P, q32, off, dx, dev, a.shape)
    shape = None
    if a.shape:
        w_, b_ = (int(x) for x in a.shape.split(","))
        shape = {"face_waves": w_, "face_blocks": b_}
    elif a.tuned:
        from paper_2207_08500_amd import autotune
        prob = native.Problem(native.EULER1D, native.FP16, native.SEL_MLP, native.TRANSMISSIVE, off,
                              dx, device=dev)
        shape = autotune.tuned(prob, native.Mlp(torch.as_tensor(P, device=dev),
                                                recheck_margin=MARGIN[native.FP16]),
                               q32, prob.workspace(dev))[0]
        torch.cuda.synchronize()
    print("workload %s%s, launch shape %s" % (a.workload, ", density wave in every other problem"
                                              if a.perturb_odd else "", shape), flush=True)
    for prec in (native.FP16, native.BF16):
        mlp = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=MARGIN[prec])
        prob = native.Problem(native.EULER1D, prec, native.SEL_MLP, native.TRANSMISSIVE, off, dx,
                              device=dev)
        prob.set_tuning(shape)
        ws = prob.workspace(dev)
        r = torch.zeros_like(q32)
        native.neno6_rhs(prob, mlp, q32, r, ws)  # builds the face map
        torch.cuda.synchronize()
        prob.flags = native.KEEP_MAP             # later calls launch only the fused kernel
        for _ in range(a.reps):
            native.neno6_rhs(prob, mlp, q32, r, ws)
        torch.cuda.synchronize()
    if not a.no_fp64:
        mlp = native.Mlp(torch.as_tensor(P, device=dev))
        prob = native.Problem(native.EULER1D, native.FP64, native.SEL_MLP, native.TRANSMISSIVE,
                              off, dx, device=dev)
        q64 = q32.double().contiguous()
        native.neno6_rhs(prob, mlp, q64, torch.zeros_like(q64), prob.workspace(dev))
        torch.cuda.synchronize()
    # calibration: a plain copy of copy_mib MiB (reads and writes that many bytes)
    n = a.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print("profiled: right-hand-side pass x%d (BF16, FP16; after one map-building call each), "
          "FP64 path x1, copy %d MiB" % (a.reps, a.copy_mib))


def step_replay(steps, P, q32, off, dx, dev, shape_arg=None):
    from paper_2207_08500_amd import autotune
    mlp = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=MARGIN[native.FP16])
    prob = native.Problem(native.EULER1D, native.FP16, native.SEL_MLP, native.TRANSMISSIVE, off, dx,
                          device=dev)
    ws = prob.workspace(dev)
    if shape_arg:
        w_, b_ = (int(x) for x in shape_arg.split(","))
        shape = {"face_waves": w_, "face_blocks": b_}
        prob.set_tuning(shape)
    else:
        shape = autotune.tuned(prob, mlp, q32, ws)[0]
    n = off.size - 1
    q = q32.clone()
    t = torch.zeros(n, dtype=torch.float64, device=dev)
    st = torch.zeros(n, dtype=torch.int32, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        native.neno6_step(prob, mlp, q, 0.4, 1, t, st, ws)  # builds the face map
    torch.cuda.current_stream().wait_stream(s)
    prob.flags = native.KEEP_MAP
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        native.neno6_step(prob, mlp, q, 0.4, 1, t, st, ws)
    q.copy_(q32)
    t.zero_()
    st.zero_()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    for _ in range(max(1, int(100.0 / max(e0.elapsed_time(e1), 1e-3)))):  # about 0.1 s
        g.replay()
    q.copy_(q32)
    t.zero_()
    st.zero_()
    marker = torch.zeros(1, device=dev)
    marker.fill_(1.0)  # the timed replays follow this dispatch
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    print("profiled: %d graph-replayed FP16 RK3 steps, launch shape %s, %.4f ms per step"
          % (steps, shape, e0.elapsed_time(e1) / steps))


def step_replay_2d(steps, P, dev):
    from paper_2207_08500_amd import autotune
    nx = ny = 2048
    q0 = inputs.riemann2d(inputs.BASE_SEED, nx, ny)
    q32 = torch.as_tensor(q0, dtype=torch.float32, device=dev).contiguous().reshape(-1)
    mlp = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=MARGIN[native.FP16])
    prob = native.Problem(native.EULER2D, native.FP16, native.SEL_MLP, native.TRANSMISSIVE, nx=nx,
                          ny=ny, dx2d=1.0 / nx, dy2d=1.0 / ny, device=dev)
    ws = prob.workspace(dev)
    shape = autotune.tuned(prob, mlp, q32, ws)[0]
    q = q32.clone()
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        native.neno6_step(prob, mlp, q, 0.4, 1, t, st, ws)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        native.neno6_step(prob, mlp, q, 0.4, 1, t, st, ws)
    q.copy_(q32)
    t.zero_()
    st.zero_()
    for _ in range(40):  # about 0.1 s: steady clocks
        g.replay()
    q.copy_(q32)
    t.zero_()
    st.zero_()
    marker = torch.zeros(1, device=dev)
    marker.fill_(1.0)  # the timed replays follow this dispatch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    print("profiled: %d graph-replayed 2D FP16 RK3 steps, launch shape %s, %.4f ms per step"
          % (steps, shape, e0.elapsed_time(e1) / steps))


if __name__ == "__main__":
    main()
