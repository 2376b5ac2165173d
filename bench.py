#!/usr/bin/env python3
"""Reconstructed faces/s of the NENO6 hot path on one MI355X.

Workload: 256 independent 1D Euler Riemann problems of 4000 cells each
(seeded synthetic states, gamma = 1.4, transmissive boundaries), the
6-64-32-16-8-4 classifier with oracle-trained weights.  One step = one SSP-RK3
step of the whole batch (time step from the CFL condition, three right-hand
sides: characteristic projection, Rusanov split, classifier per field and
sign, re-normalised combine, back-projection, flux difference, stage update);
ten steps are captured once in a HIP graph and replayed (one per replay when
the step counts are not multiples of ten).

Headline path: FP32 state, classifier in BF16 on MFMA with the FP32 re-check.
Also measured on the same GPU: the plain FP64 path and FP16-MFMA, the flip
rate of the BF16 labels against the FP64 labels on the same input state, the
L1 / Linf distance of the BF16 state from the FP64 state after the timed
steps, the fused face kernel alone (roofline), and the FP64 CPU oracle on a
bounded sample (cpu_baseline).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_PROBLEMS, N_CELLS, CFL = 256, 4000, 0.4
MARGIN = {2: 0.5, 3: 0.25}
PEAK_MFMA_BF16 = 2500.0  # TFLOP/s dense, MI355X
PEAK_HBM_GBS = 8000.0    # HBM3E, MI355X
# non-packed VALU lane-operations/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic VALU work per 1D Euler face outside the MFMA contractions,
# from rounded item estimates (primitives 90, Roe 40, projection + split 180,
# speeds 20, features 80, one operation per hidden activation 720, output
# bias + labels 50, combine 180, back-projection 12: 1372) and a strict
# one-operation-per-arithmetic-instruction count (1319); the value used lies
# between them, so the VALU fraction carries about +-2 %
VALU_OPS_PER_FACE = 1350
# 2D Euler face (one sweep): primitives 100, Roe average and eigenvectors 60,
# projection + split 240, speeds 30, features 104, hidden activations 960,
# output bias + labels 64, combine 240, back-projection 16
VALU_OPS_PER_FACE_2D = 1814
EVALS_PER_FACE_2D = 8
FLOP_PER_EVAL = 6208      # 2 x 3104 MAC of the 6-64-32-16-8-4 network
EVALS_PER_FACE = 6        # 3 characteristic fields x 2 split signs


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "euler1d_c2_256x4000_hbm_traffic.md")


def _traffic_record():
    """The committed FETCH_SIZE / WRITE_SIZE record of the fused kernel (HBM
    bytes per launch scaled by the copy-kernel calibration, and the launch
    shape the counters were taken with), or None when the kernel sources
    changed since the counters were taken."""
    import hashlib
    try:
        line = [ln for ln in open(TRAFFIC_RECORD) if ln.startswith("traffic-record:")][0]
        rec = json.loads(line.split(":", 1)[1])
        h = hashlib.sha256()
        for f in rec["sources"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        return rec if h.hexdigest() == rec["source_sha256"] else None
    except (OSError, IndexError, KeyError, ValueError):
        return None


def _alu(faces, k_ms, ops_per_face=VALU_OPS_PER_FACE):
    """VALU-issue roofline of the fused kernel (the binding one: see the
    counter profile): algorithmic lane-operations per launch / time against
    256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz."""
    ach = faces * ops_per_face / (k_ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "Tlane-op/s",
            "frac": ach / PEAK_VALU_TOPS, "ops_per_face": ops_per_face}


def _physical(q, off, gamma=1.4):
    """Per problem: every cell finite with positive density and pressure (a
    problem can leave that range in the last step; the solver freezes it only
    at the start of the next)."""
    import numpy as np
    rho, mom, E = q.double().reshape(3, -1).cpu().numpy()
    with np.errstate(all="ignore"):
        p = (gamma - 1.0) * (E - 0.5 * mom * mom / rho)
        good = np.isfinite(rho) & np.isfinite(p) & (rho > 0) & (p > 0)
    return np.minimum.reduceat(good.astype(np.int8), off[:-1]).astype(bool)


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 200 RK3 steps for c2, as the workload runs; "
                         "20 graph replays for c4)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 400 / 30 / 5)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", choices=("c2", "c3", "c4", "c5"), default="c2",
                    help="c2: 256 x 4000-cell batch (headline); c3: 2D Euler four-quadrant "
                         "Riemann problem on 2048 x 2048 cells; c4: 4096 uneven problems, "
                         "ten RK3 steps per graph replay, autotuned launch shapes; c5: "
                         "classifier training, 2^24 samples, batch 65536")
    a = ap.parse_args()
    if a.steps is None:
        a.steps = {"c2": 200, "c3": 20, "c4": 20, "c5": 179}[a.workload]
    if a.warmup is None:  # about 0.1 s: steady clocks
        a.warmup = {"c2": 400, "c3": 30, "c4": 5, "c5": 20}[a.workload]
    return a


def main():
    a = _args()
    if a.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2207_08500_amd import autotune, inputs, native

    native.load()
    dev = torch.device("cuda:0")
    P = np.load(os.path.join(ROOT, "tests", "golden", "neno6_mlp_trained.npy"), allow_pickle=False)
    if a.workload == "c4":
        return bench_batched(a, P, dev)
    if a.workload == "c3":
        return bench_2d(a, P, dev)
    if a.workload == "c5":
        return bench_train(a, dev)
    q0, off, dx = inputs.riemann1d_batch(inputs.BASE_SEED, (N_CELLS,) * N_PROBLEMS)
    faces_stage = int(off[-1]) + N_PROBLEMS
    faces_step = 3 * faces_stage
    q32 = torch.as_tensor(q0, dtype=torch.float32, device=dev).contiguous()
    q64_from32 = q32.double().contiguous()  # the same (FP32-rounded) state for both paths

    def make(prec, margin=0.0):
        mlp = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=margin)
        prob = native.Problem(native.EULER1D, prec, native.SEL_MLP, native.TRANSMISSIVE, off, dx,
                              device=dev)
        return mlp, prob, prob.workspace(dev)

    shapes_used = {}
    per_graph = {}

    def run_steps(prec, q_init, steps, warmup, graph=True):
        # ten RK3 steps per graph replay when both counts allow (about 1 %
        # faster than one: fewer replay boundaries), else one
        per = 10 if graph and steps % 10 == 0 and warmup % 10 == 0 else 1
        per_graph[prec] = per
        mlp, prob, ws = make(prec, MARGIN.get(prec, 0.0))
        if prec in (native.BF16, native.FP16):  # launch shapes from the autotuner (cached)
            shapes_used[prec] = autotune.tuned(prob, mlp, q_init, ws)[0]
        q = q_init.clone()
        t = torch.zeros(N_PROBLEMS, dtype=torch.float64, device=dev)
        st = torch.zeros(N_PROBLEMS, dtype=torch.int32, device=dev)

        def step():
            native.neno6_step(prob, mlp, q, CFL, per, t, st, ws)

        g = None
        if graph:
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                step()  # one eager step before capture
            torch.cuda.current_stream().wait_stream(s)
            q.copy_(q_init)
            t.zero_()
            st.zero_()
            prob.flags = native.KEEP_MAP  # the workspace holds the face map from the eager step
            try:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    step()
            except Exception as e:  # pragma: no cover - capture problems are reported
                print("graph capture failed, eager launches: %s" % e, file=sys.stderr)
                g = None
            q.copy_(q_init)
            t.zero_()
            st.zero_()
        go = g.replay if g is not None else step
        for _ in range(warmup // per):
            go()
        torch.cuda.synchronize()
        q.copy_(q_init)  # timed steps start from the initial state
        t.zero_()
        st.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps // per):
            go()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        return q, t, st, ms, wall, g is not None

    # ---- headline: BF16-MFMA ---------------------------------------------------
    qb, tb, stb, ms_b, wall_b, graphed = run_steps(native.BF16, q32, a.steps, a.warmup,
                                                   graph=not a.no_graph)
    value = faces_step * a.steps / (ms_b / 1e3)
    # ---- same GPU: FP64 plain and FP16-MFMA --------------------------------------
    k64 = max(2, a.steps // 4)
    q64, t64, st64, ms_64, _, _ = run_steps(native.FP64, q64_from32, k64, 1, graph=not a.no_graph)
    fp64_rate = faces_step * k64 / (ms_64 / 1e3)
    qh, th, sth, ms_h, _, _ = run_steps(native.FP16, q32, a.steps, 1, graph=not a.no_graph)
    fp16_rate = faces_step * a.steps / (ms_h / 1e3)
    # accuracy of the timed BF16 run against an FP64 run of the same number of steps
    q64b, t64b, st64b, _, _, _ = run_steps(native.FP64, q64_from32, a.steps, 0, graph=not a.no_graph)
    # problems whose state turned non-physical (no positivity limiter in the
    # scheme) are frozen by the solver and left out of the error norms
    okp = ((stb == 0) & (st64b == 0)).cpu().numpy() & _physical(qb, off) & _physical(q64b, off)
    frozen_b, frozen_64 = int((stb != 0).sum()), int((st64b != 0).sum())
    cell_ok = torch.as_tensor(np.repeat(okp, np.diff(off)), device=dev)
    dq = (qb.double() - q64b).abs().reshape(3, -1)[:, cell_ok]
    ref = q64b.reshape(3, -1)[:, cell_ok]
    l1 = float((dq.mean(dim=1) / ref.abs().mean(dim=1)).max())
    linf = float((dq.max(dim=1).values / ref.abs().max(dim=1).values).max())

    # ---- labels on an identical input state: BF16 (+re-check) vs FP64 ---------------
    def labels(prec, q):
        mlp, prob, ws = make(prec, MARGIN.get(prec, 0.0))
        r = torch.zeros_like(q)
        m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device=dev)
        native.neno6_rhs(prob, mlp, q, r, ws, masks_out=m)
        return m

    m64 = labels(native.FP64, q64_from32)
    mb16 = labels(native.BF16, q32)
    mh16 = labels(native.FP16, q32)
    torch.cuda.synchronize()

    def flip(ma, mb):
        x = (ma ^ mb).cpu().numpy()
        return float(np.unpackbits(x.reshape(-1, 1), axis=1).sum() / (8.0 * x.size))

    def flip_faces(ma, mb):  # share of faces with any differing label
        x = (ma ^ mb).reshape(3, -1).cpu().numpy()
        return float((x != 0).any(axis=0).mean())

    flip_b, flip_h = flip(mb16, m64), flip(mh16, m64)
    flip_face_b = flip_faces(mb16, m64)

    # ---- fused face kernel alone, BF16 (roofline) ------------------------------------
    mlp0, prob0, ws0 = make(native.BF16, 0.0)  # margin 0: exactly the fused kernel
    prob0.set_tuning(shapes_used.get(native.BF16))  # the launch shape of the timed steps
    F = torch.zeros(3 * faces_stage, dtype=torch.float32, device=dev)
    native.neno6_face_fluxes(prob0, mlp0, q32, F, ws0)  # builds the face map once
    prob0.flags = native.KEEP_MAP                      # later calls launch only the kernel
    for _ in range(2000):  # about 0.1 s: back to steady clocks after the host-side work above
        native.neno6_face_fluxes(prob0, mlp0, q32, F, ws0)
    torch.cuda.synchronize()
    # the timed launches back to back in one HIP graph (no host launch gaps
    # between them); eager launches if capture fails
    reps = 200
    kg = None
    if not a.no_graph:
        try:
            kg = torch.cuda.CUDAGraph()
            with torch.cuda.graph(kg):
                for _ in range(reps):
                    native.neno6_face_fluxes(prob0, mlp0, q32, F, ws0)
            kg.replay()
            torch.cuda.synchronize()
        except Exception as e:  # pragma: no cover - capture problems are reported
            print("kernel graph capture failed, eager launches: %s" % e, file=sys.stderr)
            kg = None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    if kg is not None:
        kg.replay()
    else:
        for _ in range(reps):
            native.neno6_face_fluxes(prob0, mlp0, q32, F, ws0)
    e1.record()
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / reps
    flop = faces_stage * EVALS_PER_FACE * FLOP_PER_EVAL
    # state in, face fluxes and masks out (FP32 state, one mask byte per face and field)
    alg_bytes = 3 * int(off[-1]) * 4 + 3 * faces_stage * 4 + 3 * faces_stage
    achieved = flop / (k_ms / 1e3) / 1e12
    trec = _traffic_record()
    traffic = int(trec["bytes_per_launch"]) if trec else None
    hbm_gbs = (traffic or alg_bytes) / (k_ms / 1e3) / 1e9
    # share of evaluations the FP32 re-check takes at the stated margin
    mlpm, probm, wsm = make(native.BF16, MARGIN[2])
    native.neno6_face_fluxes(probm, mlpm, q32, F, wsm)
    n_recheck = native.neno6_recheck_count(probm, mlpm, wsm)[0]
    recheck_frac = n_recheck / float(faces_stage * EVALS_PER_FACE)

    # ---- CPU oracle on a bounded sample ------------------------------------------------
    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        oracle.build()
        done_faces, t_cpu, p = 0, 0.0, 0
        while t_cpu < a.cpu_seconds and p < N_PROBLEMS:
            k = min(16, N_PROBLEMS - p)
            sub = q0[:, off[p]:off[p + k]]
            o_sub = off[p:p + k + 1] - off[p]
            c0 = time.perf_counter()
            oracle.euler1d_step(sub, o_sub, dx[p:p + k], CFL, 1, 1.4, oracle.BC_TRANSMISSIVE, P,
                                oracle.SEL_MLP)
            t_cpu += time.perf_counter() - c0
            done_faces += 3 * (int(o_sub[-1]) + k)
            p += k
        cpu = {"value": done_faces / t_cpu, "unit": "faces/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "%d of the %d problems, one RK3 step each (%d faces, %.1f s), FP64 C oracle"
                         % (p, N_PROBLEMS, done_faces, t_cpu)}

    out = {
        "metric": "reconstructed faces/s: plain FP64 vs BF16-MFMA NENO6 at stated flip rate/L1 error",
        "value": value,
        "unit": "faces/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_b / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "1D Euler Riemann batch: %d problems x %d cells, characteristic NENO6, "
                               "LF splitting, SSP-RK3 CFL %.1f; FP32 state, BF16-MFMA classifier, "
                               "FP32 re-check margin %.2f" % (N_PROBLEMS, N_CELLS, CFL, MARGIN[2]),
                   "faces_per_step": faces_step, "hip_graph": graphed,
                   "rk3_steps_per_graph_replay": per_graph.get(native.BF16, 1)},
        # the binding resource of the fused kernel is VALU issue (the
        # instruction-counter profile); the MFMA and HBM fractions follow
        "roofline": dict(_alu(faces_stage, k_ms), traffic=traffic,
                         traffic_launch_shape=trec.get("launch_shape") if trec else None,
                         kernel="k_fast_faces<BF16, 1D Euler>", kernel_ms=k_ms,
                         algorithmic_flop_per_launch=flop,
                         algorithmic_bytes_per_launch=alg_bytes),
        "roofline_mfma": {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_BF16,
                          "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_BF16},
        "roofline_hbm": {"bound": "hbm", "achieved": hbm_gbs, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": hbm_gbs / PEAK_HBM_GBS,
                         "bytes": "measured traffic" if traffic else "algorithmic"},
        "fp64_plain": {"value": fp64_rate, "unit": "faces/s", "ms_per_step": ms_64 / k64,
                       "steps": k64},
        "fp16_mfma": {"value": fp16_rate, "unit": "faces/s", "ms_per_step": ms_h / a.steps,
                      "flip_rate": flip_h},
        "speedup_bf16_vs_fp64": value / fp64_rate,
        "flip_rate": flip_b,
        "flip_rate_per_face": flip_face_b,
        "recheck_fraction": recheck_frac,
        "l1_rel_vs_fp64": l1,
        "linf_rel_vs_fp64": linf,
        "frozen_problems": {"bf16": frozen_b, "fp64": frozen_64, "of": N_PROBLEMS},
        "problems_in_error_norms": int(okp.sum()),
        "launch_shapes": {"bf16": shapes_used.get(native.BF16), "fp16": shapes_used.get(native.FP16)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def bench_batched(a, P, dev):
    """4096 independent 1D Euler problems, N log-uniform in [256, 16384];
    FP32 state, BF16 classifier; ten RK3 steps per HIP-graph replay with the
    autotuned launch shapes.  A step here is one replay (ten RK3 steps)."""
    import numpy as np
    import torch

    from paper_2207_08500_amd import autotune, inputs, native

    n_prob, inner = 4096, 10
    sizes = inputs.uneven_sizes(inputs.BASE_SEED, n_prob, 256, 16384)
    q0, off, dx = inputs.riemann1d_batch(inputs.BASE_SEED, sizes)
    faces_stage = int(off[-1]) + n_prob
    faces_replay = inner * 3 * faces_stage
    q32 = torch.as_tensor(q0, dtype=torch.float32, device=dev).contiguous()
    mlp = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=MARGIN[2])
    prob = native.Problem(native.EULER1D, native.BF16, native.SEL_MLP, native.TRANSMISSIVE, off, dx,
                          device=dev)
    ws = prob.workspace(dev)
    shapes, tune_ms = autotune.tuned(prob, mlp, q32, ws)
    q = q32.clone()
    t = torch.zeros(n_prob, dtype=torch.float64, device=dev)
    st = torch.zeros(n_prob, dtype=torch.int32, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        native.neno6_step(prob, mlp, q, CFL, 1, t, st, ws, stream=s)  # eager: builds the face map
    torch.cuda.current_stream().wait_stream(s)
    prob.flags = native.KEEP_MAP
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        native.neno6_step(prob, mlp, q, CFL, inner, t, st, ws)

    def reset():
        q.copy_(q32)
        t.zero_()
        st.zero_()

    reset()
    for _ in range(a.warmup):
        g.replay()
    torch.cuda.synchronize()
    reset()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    value = faces_replay * a.steps / (ms / 1e3)
    # fused face kernel alone (margin 0) with the tuned shapes
    mlp0 = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=0.0)
    F = torch.zeros(3 * faces_stage, dtype=torch.float32, device=dev)
    for _ in range(150):  # about 0.1 s: back to steady clocks after the host-side work above
        native.neno6_face_fluxes(prob, mlp0, q32, F, ws)
    torch.cuda.synchronize()
    reps = 20
    e0.record()
    for _ in range(reps):
        native.neno6_face_fluxes(prob, mlp0, q32, F, ws)
    e1.record()
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / reps
    flop = faces_stage * EVALS_PER_FACE * FLOP_PER_EVAL
    achieved = flop / (k_ms / 1e3) / 1e12
    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        oracle.build()
        pick = np.random.default_rng(3).choice(n_prob, 64, replace=False)
        sub = np.concatenate([q0[:, off[p]:off[p + 1]] for p in pick], axis=1)
        o_sub = np.concatenate([[0], np.cumsum(sizes[pick])])
        c0 = time.perf_counter()
        oracle.euler1d_step(sub, o_sub, dx[pick], CFL, 1, 1.4, oracle.BC_TRANSMISSIVE, P,
                            oracle.SEL_MLP)
        t_cpu = time.perf_counter() - c0
        n_f = 3 * (int(o_sub[-1]) + 64)
        cpu = {"value": n_f / t_cpu, "unit": "faces/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "64 random problems of the 4096 (%d cells), one RK3 step (%d faces, "
                         "%.1f s), FP64 C oracle" % (int(o_sub[-1]), n_f, t_cpu)}
    out = {
        "metric": "reconstructed faces/s: plain FP64 vs BF16-MFMA NENO6 at stated flip rate/L1 error",
        "value": value,
        "unit": "faces/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "1D Euler batch: %d problems, N log-uniform in [256, 16384] (%d cells), "
                               "FP32 state, BF16-MFMA classifier, re-check margin %.2f; one step = "
                               "one HIP-graph replay of %d SSP-RK3 steps" % (n_prob, int(off[-1]),
                                                                           MARGIN[2], inner),
                   "faces_per_step": faces_replay, "hip_graph": True, "launch_shapes": shapes,
                   "autotune_ms_per_face_pass": tune_ms},
        "roofline": dict(_alu(faces_stage, k_ms), traffic=None,
                         kernel="k_fast_faces<BF16, 1D Euler>", kernel_ms=k_ms,
                         algorithmic_flop_per_launch=flop),
        "roofline_mfma": {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_BF16,
                          "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_BF16},
        "frozen_problems": {"bf16": int((st != 0).sum()), "of": n_prob},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def bench_2d(a, P, dev):
    """2D Euler, four-quadrant Riemann problem on 2048 x 2048 cells
    (transmissive), FP32 state, BF16 classifier with the FP32 re-check; one
    step = one SSP-RK3 step (x and y sweeps in each stage), HIP graph."""
    import numpy as np
    import torch

    from paper_2207_08500_amd import autotune, inputs, native

    nx = ny = 2048
    q0 = inputs.riemann2d(inputs.BASE_SEED, nx, ny)
    q32 = torch.as_tensor(q0, dtype=torch.float32, device=dev).contiguous().reshape(-1)
    q64_from32 = q32.double().contiguous()

    def make(prec):
        mlp = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=MARGIN.get(prec, 0.0))
        prob = native.Problem(native.EULER2D, prec, native.SEL_MLP, native.TRANSMISSIVE, nx=nx,
                              ny=ny, dx2d=1.0 / nx, dy2d=1.0 / ny, device=dev)
        return mlp, prob, prob.workspace(dev)

    faces_stage = (nx + 1) * ny + nx * (ny + 1)
    faces_step = 3 * faces_stage
    shapes = {}

    def run(prec, q_init, steps, warmup):
        mlp, prob, ws = make(prec)
        if prec in (native.BF16, native.FP16):
            shapes[prec] = autotune.tuned(prob, mlp, q_init, ws)[0]
        q = q_init.clone()
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            native.neno6_step(prob, mlp, q, CFL, 1, t, st, ws)
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            native.neno6_step(prob, mlp, q, CFL, 1, t, st, ws)
        for _ in range(warmup):
            g.replay()
        q.copy_(q_init)
        t.zero_()
        st.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        return q, t, st, e0.elapsed_time(e1)

    qb, tb, stb, ms_b = run(native.BF16, q32, a.steps, a.warmup)
    value = faces_step * a.steps / (ms_b / 1e3)
    k64 = max(2, a.steps // 4)
    _, _, _, ms_64 = run(native.FP64, q64_from32, k64, 1)
    fp64_rate = faces_step * k64 / (ms_64 / 1e3)
    q64b, t64b, st64b, _ = run(native.FP64, q64_from32, a.steps, 0)
    dq = (qb.double() - q64b).abs().reshape(4, -1)
    l1 = float((dq.mean(dim=1) / q64b.reshape(4, -1).abs().mean(dim=1)).max())

    def labels(prec, q):
        mlp, prob, ws = make(prec)
        r = torch.zeros_like(q)
        m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device=dev)
        native.neno6_rhs(prob, mlp, q, r, ws, masks_out=m)
        return m

    x = (labels(native.BF16, q32) ^ labels(native.FP64, q64_from32)).cpu().numpy()
    # evaluations the FP32 re-check took on the initial state (both sweeps)
    mlpm, probm, wsm = make(native.BF16)
    native.neno6_face_fluxes(probm, mlpm, q32, torch.zeros(4 * faces_stage, dtype=torch.float32,
                                                            device=dev), wsm)
    recheck_frac = sum(native.neno6_recheck_count(probm, mlpm, wsm)) / float(faces_stage * EVALS_PER_FACE_2D)
    flip = float(np.unpackbits(x.reshape(-1, 1), axis=1).sum() / (8.0 * x.size))
    nfx = (nx + 1) * ny
    flip_face = float(np.concatenate([(x[:4 * nfx].reshape(4, -1) != 0).any(axis=0),
                                      (x[4 * nfx:].reshape(4, -1) != 0).any(axis=0)]).mean())
    # both sweeps of the fused face kernel alone (margin 0)
    mlp0 = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=0.0)
    _, prob0, ws0 = make(native.BF16)
    prob0.set_tuning(shapes.get(native.BF16))
    F = torch.zeros(4 * faces_stage, dtype=torch.float32, device=dev)
    for _ in range(150):  # about 0.1 s: steady clocks
        native.neno6_face_fluxes(prob0, mlp0, q32, F, ws0)
    torch.cuda.synchronize()
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        native.neno6_face_fluxes(prob0, mlp0, q32, F, ws0)
    e1.record()
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / reps
    flop = faces_stage * EVALS_PER_FACE_2D * FLOP_PER_EVAL
    achieved = flop / (k_ms / 1e3) / 1e12
    out = {
        "metric": "reconstructed faces/s: plain FP64 vs BF16-MFMA NENO6 at stated flip rate/L1 error",
        "value": value,
        "unit": "faces/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_b / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "2D Euler four-quadrant Riemann problem, %d x %d cells, transmissive, "
                               "FP32 state, BF16-MFMA classifier, re-check margin %.2f, SSP-RK3 "
                               "CFL %.1f" % (nx, ny, MARGIN[2], CFL),
                   "faces_per_step": faces_step, "hip_graph": True,
                   "launch_shapes": shapes.get(native.BF16)},
        "roofline": dict(_alu(faces_stage, k_ms, VALU_OPS_PER_FACE_2D), traffic=None,
                         kernel="k_fast_faces<BF16, 2D Euler>, x and y sweeps", kernel_ms=k_ms,
                         algorithmic_flop_per_launch=flop),
        "roofline_mfma": {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_BF16,
                          "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_BF16},
        "fp64_plain": {"value": fp64_rate, "unit": "faces/s", "ms_per_step": ms_64 / k64,
                       "steps": k64},
        "speedup_bf16_vs_fp64": value / fp64_rate,
        "flip_rate": flip,
        "flip_rate_per_face": flip_face,
        "l1_rel_vs_fp64": l1,
        "recheck_fraction": recheck_frac,
        "status": {"bf16": int(stb[0]), "fp64": int(st64b[0])},
        "cpu_baseline": None,
    }
    print(json.dumps(out))


# algorithmic work of one training sample: forward 3104 MAC, the deltas of
# layers 5..2 (32 + 128 + 512 + 2048 MAC; the input needs none) and the
# weight gradients (3104 MAC): 8928 MAC = 17 856 flop
TRAIN_FLOP_PER_SAMPLE = 2 * (3104 + 2720 + 3104)


def bench_train(a, dev):
    """C5: classifier training on 2^24 synthetic six-point samples (70 %
    training, 30 % validation), batch 65536, BF16 MFMA forward and backward
    with FP32 accumulation, FP64 master weights and Adam.  A step is one Adam
    step of one mini-batch; the timed steps run as one call over
    steps x 65536 samples of the epoch's order."""
    import numpy as np
    import torch

    from paper_2207_08500_amd import inputs, native

    n, batch = 1 << 24, 65536
    s, y = inputs.classifier_samples(inputs.BASE_SEED, n)
    n_train = int(0.7 * n)
    steps = min(a.steps, n_train // batch)
    sg = torch.as_tensor(s, dtype=torch.float32, device=dev).contiguous()
    yg = torch.as_tensor(y, device=dev).contiguous()
    P0 = inputs.mlp_init(inputs.BASE_SEED)
    Pg = torch.as_tensor(P0, device=dev).clone()
    m = torch.zeros(3228, dtype=torch.float64, device=dev)
    v = torch.zeros(3228, dtype=torch.float64, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    ws = torch.empty(native.neno6_train_workspace_size(batch), dtype=torch.uint8, device=dev)
    perm0 = torch.as_tensor(inputs.epoch_permutation(inputs.BASE_SEED, 0, n_train), device=dev)
    perm1 = torch.as_tensor(inputs.epoch_permutation(inputs.BASE_SEED, 1, n_train), device=dev)
    step = native.neno6_classifier_train(Pg, m, v, 0, sg, yg, perm0[: a.warmup * batch].contiguous(),
                                         batch, 1e-3, loss_out=loss, ws=ws)
    torch.cuda.synchronize()
    loss_warm = float(loss.item())
    idx = perm1[: steps * batch].contiguous()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    step = native.neno6_classifier_train(Pg, m, v, step, sg, yg, idx, batch, 1e-3, loss_out=loss,
                                         ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    value = steps * batch / (ms / 1e3)
    vloss = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(3228, dtype=torch.float64, device=dev)
    native.neno6_classifier_grad(Pg, sg[n_train:n_train + (1 << 20)].contiguous(),
                                 yg[n_train:n_train + (1 << 20)].contiguous(), native.FP32, g, vloss)
    torch.cuda.synchronize()
    achieved = value * TRAIN_FLOP_PER_SAMPLE / 1e12
    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        oracle.build()
        Pc, mc, vc = P0.copy(), np.zeros(3228), np.zeros(3228)
        k = 4
        c0 = time.perf_counter()
        oracle.train(Pc, mc, vc, 0, s, y, inputs.epoch_permutation(inputs.BASE_SEED, 0, n_train)[: k * batch],
                     batch, 1e-3)
        t_cpu = time.perf_counter() - c0
        cpu = {"value": k * batch / t_cpu, "unit": "samples/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "%d Adam steps of batch %d on the same samples (%.1f s), FP64 C oracle"
                         % (k, batch, t_cpu)}
    out = {
        "metric": "classifier training samples/s (BF16-MFMA forward + backward + Adam)",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "C5 classifier training: 2^24 seeded six-point samples (half smooth, "
                               "half step/kink), 70 %% training, batch %d, Adam lr 1e-3, BF16 MFMA "
                               "with FP32 accumulation, FP64 master weights" % batch,
                   "samples_per_step": batch},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_BF16,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_BF16, "traffic": None,
                     "flop_per_sample": TRAIN_FLOP_PER_SAMPLE},
        "loss": {"after_warmup": loss_warm, "after_timed_steps": float(loss.item()),
                 "validation": float(vloss.item())},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
