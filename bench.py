#!/usr/bin/env python3
"""Reconstructed faces/s of the NENO6 hot path on one MI355X.

Default workload: 4096 independent 1D Euler Riemann problems with N drawn
log-uniformly from [256, 16384] (15.6 M cells; seeded synthetic states,
gamma = 1.4, transmissive boundaries), the 6-64-32-16-8-4 classifier with
oracle-trained weights.  One step = one SSP-RK3 step of the whole batch (time
step from the CFL condition, three right-hand sides: characteristic
projection, Rusanov split, classifier per field and sign with the FP32
re-check near the cutoff, re-normalised combine, back-projection, flux
difference, stage update); ten steps are captured once in a HIP graph and
replayed.

Headline path: FP32 state, classifier layers on MFMA with FP16 operands and
FP32 accumulation, re-check margin 2x the largest FP16 logit error observed
on 2^20 training samples.  BF16 operands keep 8 significant bits against
FP16's 11, so the same rule gives BF16 a margin about nine times wider (more
evaluations go to the re-check) at the same MFMA rate; the BF16-MFMA
path is measured beside it.  Also on the same GPU: the plain FP64 path; the
labels of both reduced paths against the FP64 labels on the FP64 path's
state after the timed steps (flip rate); the L1 / Linf distance of each
reduced state from the FP64 state after the same steps; the fused kernel
alone (roofline); the FP64 CPU oracle on a bounded sample (cpu_baseline);
and the same measurements for the 256 x 4000-cell batch (nested under
"c2").

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c2|c3|c5]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CFL = 0.4
MARGINS_FILE = os.path.join(ROOT, "tests", "golden", "neno6_mlp_trained_margins.json")


def _margins():
    """Re-check margins (logit units) of the committed weights: twice the
    largest reduced-precision logit error observed on 2^20 classifier-training
    samples, keyed by precision code (2: BF16, 3: FP16)."""
    with open(MARGINS_FILE) as f:
        m = json.load(f)["margin"]
    return {2: float(m["bf16"]), 3: float(m["fp16"])}


MARGIN = _margins()
PEAK_MFMA_16 = 2500.0  # TFLOP/s dense BF16 / FP16, MI355X
PEAK_HBM_GBS = 8000.0    # HBM3E, MI355X
# non-packed VALU lane-operations/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic VALU work per 1D Euler face outside the MFMA contractions,
# from rounded item estimates (primitives 90, Roe 40, projection + split 180,
# speeds 20, features 80, one operation per hidden activation 720, output
# bias + labels 50, combine 69, back-projection 12: 1261) and a strict
# one-operation-per-arithmetic-instruction count (1208); the value used lies
# between them, so the VALU fraction carries about +-2 %.  The combine is
# counted in its table form: per reconstruction five differences, five
# products and one sum (the re-normalised combination of a selection is one
# linear stencil), plus the sum of the two split reconstructions
VALU_OPS_PER_FACE = 1235
# 2D Euler face (one sweep): primitives 100, Roe average and eigenvectors 60,
# projection + split 240, speeds 30, features 104, hidden activations 960,
# output bias + labels 64, combine 92, back-projection 16: 1666; strict count 1651
VALU_OPS_PER_FACE_2D = 1660
EVALS_PER_FACE_2D = 8
FLOP_PER_EVAL = 6208      # 2 x 3104 MAC of the 6-64-32-16-8-4 network
EVALS_PER_FACE = 6        # 3 characteristic fields x 2 split signs
METRIC = "reconstructed faces/s: plain FP64 vs BF16-MFMA NENO6 at stated flip rate/L1 error"

TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "euler1d_c4_4096_uneven_hbm_traffic.md")


def _strip_comments(text):
    """C++ source text without its comments (string and character literals
    kept) and with every run of white space collapsed to one blank."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def code_digest(paths, read=None):
    """SHA-256 over the given sources (paths relative to the repository root)
    with comments and layout removed: it changes when the code changes, not
    when a comment does."""
    import hashlib
    h = hashlib.sha256()
    for f in paths:
        if read is None:
            with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
                text = fh.read()
        else:
            text = read(f)
        h.update(_strip_comments(text).encode())
        h.update(b"\0")
    return h.hexdigest()


def _traffic_record():
    """The committed FETCH_SIZE / WRITE_SIZE record of the fused kernel on the
    4096-problem batch (HBM bytes per launch scaled by the copy-kernel
    calibration, and the launch shape the counters were taken with), or None
    when the kernel code changed since the counters were taken."""
    try:
        line = [ln for ln in open(TRAFFIC_RECORD) if ln.startswith("traffic-record:")][0]
        rec = json.loads(line.split(":", 1)[1])
        return rec if code_digest(rec["sources"]) == rec["code_sha256"] else None
    except (OSError, IndexError, KeyError, ValueError):
        return None


def _alu(faces, k_ms, ops_per_face=VALU_OPS_PER_FACE):
    """VALU-issue roofline (the binding one of the fused kernel: see the
    counter profile): algorithmic lane-operations / time against 256 CUs x 4
    SIMDs x 16 lanes x 2.4 GHz."""
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


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed RK3 steps (c4: 50, c2: 200, c3: 20; c5: Adam steps)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (about 0.1 s)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="c4: skip the nested 256 x 4000 batch")
    ap.add_argument("--no-mixed", action="store_true",
                    help="c4: skip the nested batch with a density wave in every other problem")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", choices=("c2", "c3", "c4", "c5"), default="c4",
                    help="c4: 4096 uneven 1D problems (headline); c2: 256 x 4000-cell batch; "
                         "c3: 2D Euler four-quadrant Riemann problem on 2048 x 2048 cells; "
                         "c5: classifier training, 2^24 samples, batch 65536")
    a = ap.parse_args()
    if a.steps is None:
        a.steps = {"c2": 200, "c3": 20, "c4": 50, "c5": 179}[a.workload]
    if a.warmup is None:  # about 0.1 s: steady clocks
        a.warmup = {"c2": 400, "c3": 30, "c4": 30, "c5": 20}[a.workload]
    return a


def main():
    a = _args()
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2207_08500_amd import native

    native.load()
    dev = torch.device("cuda:0")
    P = np.load(os.path.join(ROOT, "tests", "golden", "neno6_mlp_trained.npy"), allow_pickle=False)
    if a.workload == "c3":
        return bench_2d(a, P, dev)
    if a.workload == "c5":
        return bench_train(a, dev)
    out = bench_1d(a, P, dev, a.workload)
    if a.workload == "c4" and not a.no_c2:
        sub = argparse.Namespace(**vars(a))
        sub.steps, sub.warmup, sub.no_cpu_baseline = 200, 400, True
        c2 = bench_1d(sub, P, dev, "c2")
        keep = ("value", "unit", "ms_per_step", "steps", "dtype", "config", "roofline",
                "fp64_plain", "bf16_mfma", "speedup_vs_fp64", "labels", "l1_rel_vs_fp64",
                "linf_rel_vs_fp64", "frozen_problems", "end_to_end_valu_frac")
        out["c2"] = {k: c2[k] for k in keep if k in c2}
    print(json.dumps(out))


def bench_1d(a, P, dev, name):
    """One 1D Euler batch: the FP16-MFMA headline, BF16-MFMA and FP64 on the
    same GPU, labels and errors against the FP64 path, the fused kernel alone,
    the oracle on the host.  Returns the JSON-ready dict."""
    import numpy as np
    import torch

    from paper_2207_08500_amd import autotune, inputs, native

    if name == "c4":
        sizes = inputs.uneven_sizes(inputs.BASE_SEED, 4096, 256, 16384)
        label = ("1D Euler batch: 4096 Riemann problems, N log-uniform in [256, 16384] (%d cells)"
                 % int(sizes.sum()))
    else:
        sizes = np.full(256, 4000, np.int64)
        label = "1D Euler Riemann batch: 256 problems x 4000 cells"
    n_prob = sizes.size
    q0, off, dx = inputs.riemann1d_batch(inputs.BASE_SEED, sizes)
    faces_stage = int(off[-1]) + n_prob
    faces_step = 3 * faces_stage
    q32 = torch.as_tensor(q0, dtype=torch.float32, device=dev).contiguous()
    q64_from32 = q32.double().contiguous()  # the same (FP32-rounded) state for both paths

    def make(prec, margin=0.0, mode=native.RECHECK_FP32):
        mlp = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=margin, recheck_mode=mode)
        prob = native.Problem(native.EULER1D, prec, native.SEL_MLP, native.TRANSMISSIVE, off, dx,
                              device=dev)
        return mlp, prob, prob.workspace(dev)

    shapes_used = {}

    def run_steps(prec, q_init, steps, warmup, graph=True, mode=native.RECHECK_FP32):
        """steps RK3 steps from q_init after warmup untimed ones (ten per
        HIP-graph replay when both counts allow, else one)."""
        per = 10 if graph and steps % 10 == 0 and warmup % 10 == 0 else 1
        mlp, prob, ws = make(prec, MARGIN.get(prec, 0.0), mode)
        if prec in (native.BF16, native.FP16):  # launch shapes from the autotuner (cached)
            shapes_used[(prec, mode)] = autotune.tuned(prob, mlp, q_init, ws)[0]
        q = q_init.clone()
        t = torch.zeros(n_prob, dtype=torch.float64, device=dev)
        st = torch.zeros(n_prob, dtype=torch.int32, device=dev)

        def step():
            native.neno6_step(prob, mlp, q, CFL, per, t, st, ws)

        g = None
        if graph:
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                native.neno6_step(prob, mlp, q, CFL, 1, t, st, ws, stream=s)  # builds the face map
            torch.cuda.current_stream().wait_stream(s)
            prob.flags = native.KEEP_MAP
            try:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    step()
            except Exception as e:  # pragma: no cover - capture problems are reported
                print("graph capture failed, eager launches: %s" % e, file=sys.stderr)
                g = None
        go = g.replay if g is not None else step
        q.copy_(q_init)
        t.zero_()
        st.zero_()
        for _ in range(warmup // per):
            go()
        torch.cuda.synchronize()
        q.copy_(q_init)  # timed steps start from the initial state
        t.zero_()
        st.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps // per):
            go()
        e1.record()
        torch.cuda.synchronize()
        return q, t, st, e0.elapsed_time(e1), per, g is not None

    HEAD = native.FP16
    # ---- headline: FP16-MFMA -----------------------------------------------------
    qh, th, sth, ms_h, per_h, graphed = run_steps(HEAD, q32, a.steps, a.warmup,
                                                  graph=not a.no_graph)
    value = faces_step * a.steps / (ms_h / 1e3)
    # ---- same GPU: BF16-MFMA and the plain FP64 path ------------------------------
    qb, tb, stb, ms_b, _, _ = run_steps(native.BF16, q32, a.steps, a.warmup, graph=not a.no_graph)
    bf16_rate = faces_step * a.steps / (ms_b / 1e3)
    # FP16 operands with the optional two-part FP16 re-check
    qx, tx, stx, ms_x, _, _ = run_steps(HEAD, q32, a.steps, a.warmup, graph=not a.no_graph,
                                        mode=native.RECHECK_FP16X2)
    x2_rate = faces_step * a.steps / (ms_x / 1e3)
    k64 = 2 if name == "c4" else max(2, a.steps // 4)
    _, _, _, ms_64, _, _ = run_steps(native.FP64, q64_from32, k64, 1, graph=not a.no_graph)
    fp64_rate = faces_step * k64 / (ms_64 / 1e3)
    # the FP64 path over the timed steps: the accuracy reference
    q64b, _, st64b, _, _, _ = run_steps(native.FP64, q64_from32, a.steps, 0, graph=not a.no_graph)

    def errors(qa, sta, qref=None, stref=None):
        # problems whose state turned non-physical (no positivity limiter in
        # the scheme) are frozen by the solver and left out of the norms
        qref = q64b if qref is None else qref
        stref = st64b if stref is None else stref
        okp = ((sta == 0) & (stref == 0)).cpu().numpy() & _physical(qa, off) & _physical(qref, off)
        cell_ok = torch.as_tensor(np.repeat(okp, np.diff(off)), device=dev)
        dq = (qa.double() - qref).abs().reshape(3, -1)[:, cell_ok]
        ref = qref.reshape(3, -1)[:, cell_ok]
        return (float((dq.mean(dim=1) / ref.abs().mean(dim=1)).max()),
                float((dq.max(dim=1).values / ref.abs().max(dim=1).values).max()), int(okp.sum()))

    l1, linf, n_norm = errors(qh, sth)
    l1_b, linf_b, _ = errors(qb, stb)
    l1_x, linf_x, _ = errors(qx, stx)

    # ---- labels on the evolved state: the FP64 path's state after the timed
    # steps, rounded to FP32, through the FP16 / BF16 pass (re-check on) and
    # the FP64 pass -------------------------------------------------------------------
    q_ev32 = q64b.float().contiguous()
    q_ev64 = q_ev32.double().contiguous()

    def labels(prec, q, margin, mode=native.RECHECK_FP32):
        mlp, prob, ws = make(prec, margin, mode)
        r = torch.zeros_like(q)
        m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device=dev)
        n_re = 0
        if prec >= native.BF16:
            # evaluations re-checked as in a step (no labels requested: faces
            # with six equal cells skip it, their flux does not depend on it)
            native.neno6_rhs(prob, mlp, q, r, ws)
            n_re = native.neno6_recheck_count(prob, mlp, ws)[0]
        native.neno6_rhs(prob, mlp, q, r, ws, masks_out=m)
        torch.cuda.synchronize()
        return m, n_re

    m64, _ = labels(native.FP64, q_ev64, 0.0)
    mh16, re_h = labels(native.FP16, q_ev32, MARGIN[3])
    mh0, _ = labels(native.FP16, q_ev32, 0.0)
    mb16, re_b = labels(native.BF16, q_ev32, MARGIN[2])
    mx16, _ = labels(native.FP16, q_ev32, MARGIN[3], native.RECHECK_FP16X2)
    mb0, _ = labels(native.BF16, q_ev32, 0.0)

    def flip(ma, mb):
        x = (ma ^ mb).cpu().numpy()
        return float(np.unpackbits(x.reshape(-1, 1), axis=1).sum() / (8.0 * x.size))

    def flip_faces(ma, mb):  # share of faces with any differing label
        x = (ma ^ mb).reshape(3, -1).cpu().numpy()
        return float((x != 0).any(axis=0).mean())

    n_evals = faces_stage * EVALS_PER_FACE

    # ---- the same batch with a density wave in every other problem (the
    # Riemann states of the headline and perturbed ones): smooth regions
    # instead of constant states -------------------------------------------------------
    mixed = None
    if name == "c4" and not a.no_mixed:
        qm0, _, _ = inputs.riemann1d_batch(inputs.BASE_SEED, sizes, perturb="odd")
        qm32 = torch.as_tensor(qm0, dtype=torch.float32, device=dev).contiguous()
        qmh, _, stmh, ms_mh, _, _ = run_steps(HEAD, qm32, a.steps, a.warmup, graph=not a.no_graph)
        qmb, _, stmb, ms_mb, _, _ = run_steps(native.BF16, qm32, a.steps, a.warmup,
                                              graph=not a.no_graph)
        qm64, _, stm64, _, _, _ = run_steps(native.FP64, qm32.double().contiguous(), a.steps, 0,
                                            graph=not a.no_graph)
        l1_m, linf_m, n_m = errors(qmh, stmh, qm64, stm64)
        l1_mb, linf_mb, _ = errors(qmb, stmb, qm64, stm64)
        qm_ev32 = qm64.float().contiguous()
        mm64, _ = labels(native.FP64, qm_ev32.double().contiguous(), 0.0)
        mmh, re_mh = labels(native.FP16, qm_ev32, MARGIN[3])
        mmb, re_mb = labels(native.BF16, qm_ev32, MARGIN[2])
        mixed = {"workload": "the same 4096 problems, those of odd index with the density "
                             "multiplied by 1 + 0.2 sin(2 pi k x), k in 1..8",
                 "value": faces_step * a.steps / (ms_mh / 1e3), "unit": "faces/s",
                 "ms_per_step": ms_mh / a.steps, "l1_rel_vs_fp64": l1_m,
                 "linf_rel_vs_fp64": linf_m, "flip_rate": flip(mmh, mm64),
                 "recheck_fraction": re_mh / float(n_evals),
                 "bf16_mfma": {"value": faces_step * a.steps / (ms_mb / 1e3), "unit": "faces/s",
                               "ms_per_step": ms_mb / a.steps, "l1_rel_vs_fp64": l1_mb,
                               "linf_rel_vs_fp64": linf_mb, "flip_rate": flip(mmb, mm64),
                               "recheck_fraction": re_mb / float(n_evals)},
                 "frozen_problems": {"fp16": int((stmh != 0).sum()),
                                     "bf16": int((stmb != 0).sum()),
                                     "fp64": int((stm64 != 0).sum())},
                 "problems_in_error_norms": n_m}

    lab = {"state": "FP64 path after the %d timed RK3 steps, rounded to FP32" % a.steps,
           "flip_rate_fp16": flip(mh16, m64), "flip_rate_per_face_fp16": flip_faces(mh16, m64),
           "flip_rate_fp16_without_recheck": flip(mh0, m64),
           "flip_rate_bf16": flip(mb16, m64), "flip_rate_per_face_bf16": flip_faces(mb16, m64),
           "flip_rate_bf16_without_recheck": flip(mb0, m64),
           "flip_rate_fp16_two_part_recheck": flip(mx16, m64),
           "recheck_margin": {"fp16": MARGIN[3], "bf16": MARGIN[2]},
           # the overlap face of two 64-face tiles is counted by both
           "recheck_fraction_fp16": re_h / float(n_evals),
           "recheck_fraction_bf16": re_b / float(n_evals)}

    # ---- fused kernel alone: the right-hand-side pass as inside the step, on
    # the states of the headline trajectory (every tenth step of the timed ones:
    # the classifier's work and the share of flat stencils change as the
    # solution evolves) --------------------------------------------------------------
    mlpk, probk, wsk = make(HEAD, MARGIN[HEAD])
    probk.set_tuning(shapes_used.get((HEAD, native.RECHECK_FP32)))  # shape of the timed steps
    snaps = [q32.clone()]
    qs = q32.clone()
    ts = torch.zeros(n_prob, dtype=torch.float64, device=dev)
    sts = torch.zeros(n_prob, dtype=torch.int32, device=dev)
    for k in range(0, a.steps, 10):
        native.neno6_step(probk, mlpk, qs, CFL, min(10, a.steps - k), ts, sts, wsk)
        snaps.append(qs.clone())
    torch.cuda.synchronize()
    r = torch.zeros_like(q32)
    native.neno6_rhs(probk, mlpk, q32, r, wsk)  # builds the face map once
    probk.flags = native.KEEP_MAP               # later calls launch only the kernel
    reps = 200 if name == "c2" else 20
    qk = torch.empty_like(q32)

    def launches():
        for _ in range(reps):
            native.neno6_rhs(probk, mlpk, qk, r, wsk)

    qk.copy_(snaps[0])
    for _ in range(10):  # about 0.1 s: back to steady clocks
        launches()
    torch.cuda.synchronize()
    kg = None
    if not a.no_graph:
        try:  # the launches back to back in one HIP graph (no host gaps between them)
            kg = torch.cuda.CUDAGraph()
            with torch.cuda.graph(kg):
                launches()
            kg.replay()
            torch.cuda.synchronize()
        except Exception as e:  # pragma: no cover
            print("kernel graph capture failed, eager launches: %s" % e, file=sys.stderr)
            kg = None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k_each = []
    for sq in snaps:
        qk.copy_(sq)
        e0.record()
        if kg is not None:
            kg.replay()
        else:
            launches()
        e1.record()
        torch.cuda.synchronize()
        k_each.append(e0.elapsed_time(e1) / reps)
    k_ms = float(np.mean(k_each))
    flop = faces_stage * EVALS_PER_FACE * FLOP_PER_EVAL
    # state in, right-hand side out (FP32)
    alg_bytes = 2 * 3 * int(off[-1]) * 4
    achieved = flop / (k_ms / 1e3) / 1e12
    trec = _traffic_record() if name == "c4" else None
    traffic = int(trec["bytes_per_launch"]) if trec else None

    # ---- CPU oracle on a bounded sample ------------------------------------------------
    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        oracle.build()

        def oracle_rate(threads, budget, max_problems):
            oracle.set_num_threads(threads)
            pick = np.random.default_rng(3).permutation(n_prob)
            done, t_cpu, used = 0, 0.0, 0
            while t_cpu < budget and used < min(max_problems, n_prob):
                k = min(16 if threads > 1 else 2, n_prob - used)
                pp = np.sort(pick[used:used + k])
                sub = np.concatenate([q0[:, off[p]:off[p + 1]] for p in pp], axis=1)
                o_sub = np.concatenate([[0], np.cumsum(sizes[pp])])
                c0 = time.perf_counter()
                oracle.euler1d_step(sub, o_sub, dx[pp], CFL, 1, 1.4, oracle.BC_TRANSMISSIVE, P,
                                    oracle.SEL_MLP)
                t_cpu += time.perf_counter() - c0
                done += 3 * (int(o_sub[-1]) + k)
                used += k
            return done / t_cpu, used, done, t_cpu

        ncpu = os.cpu_count() or 1
        v_all, used, done, t_all = oracle_rate(ncpu, a.cpu_seconds, 256)
        v_one, used1, done1, t_one = oracle_rate(1, a.cpu_seconds / 4, 16)
        oracle.set_num_threads(ncpu)
        cpu = {"value": v_all, "unit": "faces/s", "cores": ncpu, "kind": "oracle",
               "cpu_model": _cpu_model(), "nproc": ncpu,
               "sample": "%d random problems of the %d, one RK3 step each (%d faces, %.1f s), "
                         "FP64 C oracle, OpenMP over problems" % (used, n_prob, done, t_all),
               "single_thread": {"value": v_one, "unit": "faces/s",
                                 "sample": "%d problems, one RK3 step (%d faces, %.1f s)"
                                           % (used1, done1, t_one)}}

    e2e = value * VALU_OPS_PER_FACE / 1e12 / PEAK_VALU_TOPS
    return {
        "metric": METRIC,
        "value": value,
        "unit": "faces/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_h / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16",
        "data": "synthetic",
        "config": {"workload": "%s; characteristic NENO6, LF splitting, SSP-RK3 CFL %.1f; FP32 "
                               "state, classifier on MFMA with FP16 operands and FP32 "
                               "accumulation, FP32 re-check margin %.2f (BF16 operands: "
                               "bf16_mfma, margin %.2f; the optional two-part FP16 re-check: "
                               "fp16_two_part_recheck)" % (label, CFL, MARGIN[3], MARGIN[2]),
                   "faces_per_step": faces_step, "hip_graph": graphed,
                   "rk3_steps_per_graph_replay": per_h,
                   "launch_shapes": {"fp16": shapes_used.get((native.FP16, native.RECHECK_FP32)),
                                     "bf16": shapes_used.get((native.BF16, native.RECHECK_FP32))}},
        # the binding resource of the fused kernel is VALU issue (the
        # instruction-counter profile); the MFMA and HBM fractions follow
        "roofline": dict(_alu(faces_stage, k_ms), traffic=traffic,
                         traffic_launch_shape=trec.get("launch_shape") if trec else None,
                         kernel="k_euler1d<FP16> (fused faces, re-check, flux difference; "
                                "right-hand-side output)", kernel_ms=k_ms,
                         kernel_ms_by_step={str(10 * i): v for i, v in enumerate(k_each)},
                         algorithmic_flop_per_launch=flop,
                         algorithmic_bytes_per_launch=alg_bytes),
        "end_to_end_valu_frac": e2e,
        "roofline_mfma": {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_16,
                          "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_16},
        "roofline_hbm": {"bound": "hbm",
                         "achieved": (traffic or alg_bytes) / (k_ms / 1e3) / 1e9,
                         "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": (traffic or alg_bytes) / (k_ms / 1e3) / 1e9 / PEAK_HBM_GBS,
                         "bytes": "measured traffic" if traffic else "algorithmic"},
        "fp64_plain": {"value": fp64_rate, "unit": "faces/s", "ms_per_step": ms_64 / k64,
                       "steps": k64},
        "bf16_mfma": {"value": bf16_rate, "unit": "faces/s", "ms_per_step": ms_b / a.steps,
                      "recheck_margin": MARGIN[2], "l1_rel_vs_fp64": l1_b,
                      "linf_rel_vs_fp64": linf_b, "speedup_vs_fp64": bf16_rate / fp64_rate},
        "fp16_two_part_recheck": {"value": x2_rate, "unit": "faces/s",
                                  "ms_per_step": ms_x / a.steps, "recheck_margin": MARGIN[3],
                                  "flip_rate": lab["flip_rate_fp16_two_part_recheck"],
                                  "l1_rel_vs_fp64": l1_x, "linf_rel_vs_fp64": linf_x,
                                  "vs_fp32_recheck": x2_rate / value},
        "speedup_vs_fp64": value / fp64_rate,
        "labels": lab,
        "flip_rate": lab["flip_rate_fp16"],
        "l1_rel_vs_fp64": l1,
        "linf_rel_vs_fp64": linf,
        "frozen_problems": {"fp16": int((sth != 0).sum()), "bf16": int((stb != 0).sum()),
                            "fp64": int((st64b != 0).sum()), "of": n_prob},
        "problems_in_error_norms": n_norm,
        "perturbed_half": mixed,
        "cpu_baseline": cpu,
    }


def bench_2d(a, P, dev):
    """2D Euler, four-quadrant Riemann problem on 2048 x 2048 cells
    (transmissive), FP32 state, classifier on FP16 MFMA with the FP32
    re-check; one step = one SSP-RK3 step (x and y sweeps in each stage), HIP
    graph."""
    import numpy as np
    import torch

    from paper_2207_08500_amd import autotune, inputs, native

    nx = ny = 2048
    q0 = inputs.riemann2d(inputs.BASE_SEED, nx, ny)
    q32 = torch.as_tensor(q0, dtype=torch.float32, device=dev).contiguous().reshape(-1)
    q64_from32 = q32.double().contiguous()

    def make(prec, mode=native.RECHECK_FP32):
        mlp = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=MARGIN.get(prec, 0.0),
                         recheck_mode=mode)
        prob = native.Problem(native.EULER2D, prec, native.SEL_MLP, native.TRANSMISSIVE, nx=nx,
                              ny=ny, dx2d=1.0 / nx, dy2d=1.0 / ny, device=dev)
        return mlp, prob, prob.workspace(dev)

    faces_stage = (nx + 1) * ny + nx * (ny + 1)
    faces_step = 3 * faces_stage
    shapes = {}

    def run(prec, q_init, steps, warmup, mode=native.RECHECK_FP32):
        mlp, prob, ws = make(prec, mode)
        if prec == native.FP16:
            shapes[(prec, mode)] = autotune.tuned(prob, mlp, q_init, ws)[0]
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

    qb, tb, stb, ms_b = run(native.FP16, q32, a.steps, a.warmup)
    value = faces_step * a.steps / (ms_b / 1e3)
    k64 = max(2, a.steps // 4)
    _, _, _, ms_64 = run(native.FP64, q64_from32, k64, 1)
    fp64_rate = faces_step * k64 / (ms_64 / 1e3)
    qx, _, stx, ms_x = run(native.FP16, q32, a.steps, a.warmup, native.RECHECK_FP16X2)
    x2_rate = faces_step * a.steps / (ms_x / 1e3)
    q64b, t64b, st64b, _ = run(native.FP64, q64_from32, a.steps, 0)

    def l1_of(qa):
        dq = (qa.double() - q64b).abs().reshape(4, -1)
        return float((dq.mean(dim=1) / q64b.reshape(4, -1).abs().mean(dim=1)).max())

    l1, l1_x = l1_of(qb), l1_of(qx)

    def labels(prec, q, mode=native.RECHECK_FP32):
        mlp, prob, ws = make(prec, mode)
        r = torch.zeros_like(q)
        m = torch.zeros(prob.mask_count(), dtype=torch.uint8, device=dev)
        native.neno6_rhs(prob, mlp, q, r, ws, masks_out=m)
        return m

    m64 = labels(native.FP64, q64_from32)
    x = (labels(native.FP16, q32) ^ m64).cpu().numpy()
    xx = (labels(native.FP16, q32, native.RECHECK_FP16X2) ^ m64).cpu().numpy()
    # evaluations the re-check took on the initial state (both sweeps)
    mlpm, probm, wsm = make(native.FP16)
    native.neno6_face_fluxes(probm, mlpm, q32, torch.zeros(4 * faces_stage, dtype=torch.float32,
                                                            device=dev), wsm)
    recheck_frac = sum(native.neno6_recheck_count(probm, mlpm, wsm)) / float(faces_stage * EVALS_PER_FACE_2D)
    flip = float(np.unpackbits(x.reshape(-1, 1), axis=1).sum() / (8.0 * x.size))
    flip_x = float(np.unpackbits(xx.reshape(-1, 1), axis=1).sum() / (8.0 * xx.size))
    nfx = (nx + 1) * ny
    flip_face = float(np.concatenate([(x[:4 * nfx].reshape(4, -1) != 0).any(axis=0),
                                      (x[4 * nfx:].reshape(4, -1) != 0).any(axis=0)]).mean())
    # both sweeps of the fused face kernel alone (margin 0)
    mlp0 = native.Mlp(torch.as_tensor(P, device=dev), recheck_margin=0.0)
    _, prob0, ws0 = make(native.FP16)
    prob0.set_tuning(shapes.get((native.FP16, native.RECHECK_FP32)))
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
        "metric": METRIC,
        "value": value,
        "unit": "faces/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_b / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16",
        "data": "synthetic",
        "config": {"workload": "2D Euler four-quadrant Riemann problem, %d x %d cells, transmissive, "
                               "FP32 state, FP16-MFMA classifier, FP32 re-check margin %.2f (the "
                               "optional two-part FP16 re-check: fp16_two_part_recheck), SSP-RK3 "
                               "CFL %.1f" % (nx, ny, MARGIN[3], CFL),
                   "faces_per_step": faces_step, "hip_graph": True,
                   "launch_shapes": shapes.get((native.FP16, native.RECHECK_FP32))},
        "roofline": dict(_alu(faces_stage, k_ms, VALU_OPS_PER_FACE_2D), traffic=None,
                         kernel="k_fast_faces<FP16, 2D Euler>, x and y sweeps", kernel_ms=k_ms,
                         algorithmic_flop_per_launch=flop),
        "roofline_mfma": {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_16,
                          "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_16},
        "fp64_plain": {"value": fp64_rate, "unit": "faces/s", "ms_per_step": ms_64 / k64,
                       "steps": k64},
        "fp16_two_part_recheck": {"value": x2_rate, "unit": "faces/s",
                                  "ms_per_step": ms_x / a.steps, "flip_rate": flip_x,
                                  "l1_rel_vs_fp64": l1_x, "vs_fp32_recheck": x2_rate / value,
                                  "status": int(stx[0])},
        "speedup_vs_fp64": value / fp64_rate,
        "flip_rate": flip,
        "flip_rate_per_face": flip_face,
        "l1_rel_vs_fp64": l1,
        "recheck_fraction": recheck_frac,
        "status": {"fp16": int(stb[0]), "fp64": int(st64b[0])},
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
    # the samples are generated on the device (seeded, counter-based)
    native.neno6_classifier_samples(inputs.BASE_SEED, 0, 1024)  # warm the kernel
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record()
    sg, yg = native.neno6_classifier_samples(inputs.BASE_SEED, 0, n)
    g1.record()
    torch.cuda.synchronize()
    gen_rate = n / (g0.elapsed_time(g1) / 1e3)
    n_train = int(0.7 * n)
    steps = min(a.steps, n_train // batch)
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
        s_h, y_h, _ = inputs.classifier_samples_philox(inputs.BASE_SEED, 0, k * batch)
        c0 = time.perf_counter()
        oracle.train(Pc, mc, vc, 0, s_h.astype(np.float64), y_h, np.arange(k * batch), batch, 1e-3)
        t_cpu = time.perf_counter() - c0
        cpu = {"value": k * batch / t_cpu, "unit": "samples/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "%d Adam steps of batch %d on the first %d samples (%.1f s), FP64 C "
                         "oracle" % (k, batch, k * batch, t_cpu)}
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
        "config": {"workload": "C5 classifier training: 2^24 seeded six-point samples generated on "
                               "the device (half smooth, half step/kink), 70 %% training, batch %d, "
                               "Adam lr 1e-3, BF16 MFMA with FP32 accumulation, FP64 master "
                               "weights" % batch,
                   "samples_per_step": batch},
        "sample_generation": {"value": gen_rate, "unit": "samples/s",
                              "what": "Philox4x32-10 counter-based generator, FP64 recipe"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_16,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_16, "traffic": None,
                     "flop_per_sample": TRAIN_FLOP_PER_SAMPLE},
        "loss": {"after_warmup": loss_warm, "after_timed_steps": float(loss.item()),
                 "validation": float(vloss.item())},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
