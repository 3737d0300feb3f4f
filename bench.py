#!/usr/bin/env python3
"""Benchmark of the CoFEM E-step hot path on one MI355X.

A step is one full CoFEM solve of the workload: T_em EM iterations of
Algorithm 1 from alpha = 1 (E-step by multi-right-hand-side CG, diagonal
estimate, M-step), on inputs already resident in HBM.  The reported value is
EM iterations per second over the timed steps.

Default workload: the 1024 x 1024 circular convolution with 9x9 taps (D =
2^20, K = 16, beta = 1e4, eps = 1e-5, U = 400, T_em = 30).  The headline form
is the learned start (a network trained on the GPU by the library's kernels
on EM iterates of other seeds predicts each E-step's start; Jacobi-
preconditioned CG from there); the non-learned control (the previous iterate
as the start, Jacobi) and plain float32 CG are timed the same way under
"forms".  Each form's mean after the first m EM iterations is compared with a
float64 oracle run of the control's algorithm (NMSE, "oracle_trajectory");
that run is the CPU sample too.  The same line carries, under "secondary",
the dense 4096 x 16384 workload: bf16 refinement vs float32 CG, both warm-
started, and float32 CG from zero; under "time_to_target", the DCT protocol of
Sec. 4.2 (EM iterations and GPU time to an NRMSE of 2% at D = 2^18) and where
the library's EM-level stop rule ends the same run.

Besides the throughput line the JSON carries:
  roofline      the dominant operator kernel against HBM: algorithmic bytes
                per launch / mean launch time, the times from HIP events the
                library records on its stream around the launches of every
                n-th CG iteration during the timed steps (--timing-every n),
                with the counter-measured HBM bytes per launch when a stored
                rocprofv3 summary matches the current kernel source; for the
                stencil also its flops against the fp32 vector ALU;
  cpu_baseline  the float64 oracle timed on this host on a bounded sample,
                scaled to EM iterations per second at the GPU run's CG counts
                (with a one-thread figure and the host's CPU model);
  parity        (dense) relative errors of the first GPU step vs the oracle.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "EM iters/sec at fixed NMSE vs FP64 oracle; bf16+learned vs plain FP32 CG"
HBM_PEAK_GBS = 8000.0
# MI355X fp32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2
# (packed FP32) x 2.4 GHz.  The library is built without packed FP32
# instructions, so its own issue ceiling is half of this (78.6 TFLOP/s).
FP32_VALU_PEAK_TFS = 157.3
FP32_VALU_ISSUE_TFS = 78.6


def algorithmic_flops(p, which):
    """Flops one launch of the fused conv operator pass must do: the k x k
    stencil of Phi and of Phi^T (one FMA per tap each) on every pixel of the
    K + 1 columns.  The halo recomputation and the alpha/dot epilogue are not
    counted."""
    k = p.taps.shape[0]
    return 2 * 2 * k * k * p.D * (p.K + 1)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(p, which, phi_bytes=4):
    """Bytes one launch must move at minimum: the dictionary once (4 bytes an
    entry in float32, 2 in bfloat16) plus the skinny operands it is contracted
    with (K probe columns float32, the mean column float64)."""
    K, N, D = p.K, p.N, p.D
    col = 4 * K + 8
    if p.kind == "dense":
        if which == "pass1":   # W = Phi P: Phi, P in, W out
            return phi_bytes * N * D + D * col + N * col
        # pass 2: Phi, W in; P, R, alpha in; Q out
        return phi_bytes * N * D + N * col + 3 * D * col + 4 * D
    # conv fused iteration: p, r, q, x and alpha in; x, r, p, q out (taps
    # negligible; the halo re-reads are not counted)
    return 8 * D * col + 4 * D


KERNEL_NAMES = {"dense": {"pass1": "k_dense_pass1", "pass2": "k_dense_pass2", "update": "k_dense_update"},
                "dct": {"pass1": "k_dct_rows_in", "pass2": "k_dct_mid", "update": "k_dct_rows_out"},
                "dense_bf16_ir": {"pass1": "k_dense16_pass1", "pass2": "k_dense16_pass2", "update": "k_dense_update"},
                "conv": {"pass1": "k_conv_fused"}, "conv_ws": {"pass1": "k_conv_ws"}}
FORMS = {"fp32": "fp32 probes + fp64 mean column",
         "fp32_warm": "fp32 Jacobi-preconditioned CG started from the previous mean and diagonal estimate (fp64 "
                      "mean column)",
         "bf16_ir": "bf16 Phi inner Jacobi-preconditioned CG + float32-Phi iterative refinement (fp64 mean column), "
                    "started from the "
                    "previous mean and diagonal estimate",
         "control": "fp32 CG started from the previous mean and diagonal estimate, Jacobi-preconditioned",
         "learned": "fp32 CG started from a learned prediction, Jacobi-preconditioned"}
SPECTRAL_NOTE = "; the first E-step (alpha = 1) starts from the 2D-DFT solve of its block-circulant system"
DENSE_FORM_ORDER = ("bf16_ir", "fp32_warm", "fp32")
FORMS_DCT = {"fp32": "inverse-DCT + mask dictionary, plain fp32 CG + fp64 mean column",
             "control": "inverse-DCT + mask dictionary, fp32 CG started from the previous mean and diagonal "
                        "estimate, Jacobi-preconditioned, fp64 mean column"}
KERNEL_SOURCES = {"dense": ("paper_2202_12808_amd/csrc/kernels_dense.hip", "paper_2202_12808_amd/csrc/cofem_internal.h"),
                  "dense_bf16_ir": ("paper_2202_12808_amd/csrc/kernels_dense_bf16.hip",
                                    "paper_2202_12808_amd/csrc/cofem_internal.h"),
                  "conv": ("paper_2202_12808_amd/csrc/kernels_conv.hip", "paper_2202_12808_amd/csrc/conv_tile.h",
                           "paper_2202_12808_amd/csrc/cofem_internal.h"),
                  "conv_ws": ("paper_2202_12808_amd/csrc/kernels_conv_ws.hip", "paper_2202_12808_amd/csrc/conv_tile.h",
                              "paper_2202_12808_amd/csrc/cofem_internal.h"),
                  "dct": ("paper_2202_12808_amd/csrc/kernels_dct.hip", "paper_2202_12808_amd/csrc/cofem_internal.h")}


def kernel_source_sha256(kind):
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(kind, kernel, workload):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    kept in profiles/, or None when there is none or the kernel source has
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_sha256(kind):
        log(f"{path}: kernel source changed since the counters were taken; traffic reported as null")
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calibration_copies(args, dev):
    """--calibration-copy-mib m: three plain device copies of m MiB before the
    workload, whose FETCH_SIZE and WRITE_SIZE counters scale the kernels' (a
    copy reads and writes exactly 2^20 m bytes)."""
    if args.calibration_copy_mib <= 0:
        return
    import torch

    n = args.calibration_copy_mib << 18
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"calibration: 3 copies of {4 * n} bytes")
    del src, dst


def train_predictor(p, dev, train_size=256, seeds=(1000, 1001, 1002), em_iters=None, epochs=20, lr=1e-3,
                    spectral=True):
    """Trains the learned form's network on EM iterates of `seeds` (disjoint
    from the evaluation seed) at train_size^2 with the workload's kernel law,
    beta, K and tolerance (warm-started Jacobi solves give the targets), then
    returns a network of the workload's image size with those parameters."""
    import torch

    from paper_2202_12808_amd import learned as LD
    from paper_2202_12808_amd import synth
    from paper_2202_12808_amd.cofem import CoFEM, CoFEMNet

    t0 = time.perf_counter()
    hs = min(train_size, p.H)
    ws = min(train_size, p.W)
    small = CoFEMNet(hs, ws, seed=7)

    def mk(sd):
        q = synth.conv_problem(hs, ws, p.taps.shape[0], rho=float(round(p.z.astype(bool).mean(), 4)), beta=p.beta,
                               K=p.K, tol=p.tol, max_iter=p.max_iter, seed=sd, name="train")
        return CoFEM.conv(torch.from_numpy(q.taps).to(dev), torch.from_numpy(q.y).to(dev), q.H, q.W, q.beta, q.K,
                          tol=q.tol, max_iter=q.max_iter, seed=sd, jacobi=True, warm_start=True,
                          spectral_start=spectral)

    # every EM iteration of the workload's run: late iterations, where the
    # previous iterate is already a good start, must be learned too
    samples = LD.collect_samples(mk, seeds, em_iters or p.T_em, small)
    before = LD.mean_loss(small, samples)
    hist = LD.train(small, samples, epochs=epochs, lr=lr)
    after = LD.mean_loss(small, samples)
    net = small
    if (hs, ws) != (p.H, p.W):
        net = CoFEMNet(p.H, p.W)
        net.set_params(small.get_params())
        small.close()
    info = {"train_image": [hs, ws], "seeds": list(seeds), "em_iters": em_iters or p.T_em,
            "samples": len(samples), "epochs": epochs,
            "loss_before": round(before, 6), "loss_after": round(after, 6),
            "seconds": round(time.perf_counter() - t0, 2)}
    log(f"learned predictor trained: {info}")
    return net, info


def run_batched(args):
    """The batched workload: 64 dense problems (D_i = 4 U{256..4096}, N_i =
    D_i/4, bf16 dictionaries) advanced together; a step is T_em EM iterations
    of the whole batch from alpha = 1."""
    import numpy as np
    import torch

    from paper_2202_12808_amd import synth
    from paper_2202_12808_amd.cofem import CoFEMBatch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    probs = synth.batched_64(0)
    p0 = probs[0]
    T_em = args.em_iters or p0.T_em
    n = len(probs)
    sizes = [p.D for p in probs]
    log(f"workload batched_64: {n} problems, D in [{min(sizes)}, {max(sizes)}], N = D/4, "
        f"sum N*D = {sum(p.N * p.D for p in probs):.3e}, K={p0.K} beta={p0.beta} tol={p0.tol} T_em={T_em} "
        f"(inputs generated in {time.perf_counter() - t_gen:.1f}s)")
    pairs = [(torch.from_numpy(p.phi).to(dev), torch.from_numpy(p.y).to(dev)) for p in probs]
    g = CoFEMBatch(pairs, p0.beta, p0.K, tol=p0.tol, max_iter=p0.max_iter, seed=p0.seed)
    plan = g.plan()
    log(f"autotuner: {plan['target_wgs']} workgroups per pass (candidate ms {plan['candidate_ms']})")
    ones = [torch.ones(D, dtype=torch.float32, device=dev) for D in sizes]

    def one_step():
        for i in range(n):
            g.set_alpha(i, ones[i])
        g.set_iteration(1)
        return g.em_step(T_em)

    for i in range(n):
        g.set_alpha(i, ones[i])
    g.set_iteration(1)
    first = g.em_step(1)[0]
    firsts = [[x.cpu().numpy().astype(np.float64) for x in g.posterior(i)] for i in range(n)]
    for w in range(args.warmup):
        one_step()
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = one_step()
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = args.steps * T_em / elapsed
    cg = np.array([[x["cg_iters"] for x in it] for it in st])  # T_em x n
    log(f"{value:.3f} batch EM it/s; CG iterations per EM iteration: mean over problems {cg.mean():.1f}, "
        f"max per EM iteration (the batch's critical path) mean {cg.max(axis=1).mean():.1f}")

    ms = g.time_operator(10)
    col = 4 * p0.K + 8
    b1 = sum(2 * p.N * p.D + p.D * col + p.N * col for p in probs)
    b2 = sum(2 * p.N * p.D + p.N * col + 3 * p.D * col + 4 * p.D for p in probs)
    per = {"k_batch_pass1": ms[0], "k_batch_pass2": ms[1]}
    nbytes = {"k_batch_pass1": b1, "k_batch_pass2": b2}
    dom = max(per, key=per.get)
    achieved = nbytes[dom] / (per[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                "bytes_per_launch": nbytes[dom], "ms_per_launch": round(per[dom], 5),
                "timing": "cofem_time_operator: grouped passes over all problems, back to back",
                "kernels": {k: {"ms_per_launch": round(v, 5)} for k, v in per.items()}}
    log(f"roofline: {dom} {per[dom] * 1e3:.1f} us/launch, {achieved:.0f} GB/s "
        f"({100 * achieved / HBM_PEAK_GBS:.1f}% of HBM peak)")

    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle as O
        threads = os.cpu_count()
        order = np.argsort(sizes)
        sample = [int(order[0]), int(order[n // 2]), int(order[-1])]
        t_el = 0.0
        per_elem_iter = []
        parity = {}
        for i in sample:
            p = probs[i]
            op = O.DenseOperator(synth.round_to_bf16(p.phi).astype(np.float64))
            tc0 = time.perf_counter()
            b0 = p.beta * op.apply_t(p.y.astype(np.float64))
            e = O.cofem_estep(op, b0, p.beta, np.ones(p.D), p.K, p.tol, p.max_iter, p0.seed + i, 1,
                              fixed_iters=first[i]["cg_iters"])
            a_ref, _ = O.mstep(e.mu, e.s)
            dt = time.perf_counter() - tc0
            t_el += dt
            per_elem_iter.append(dt / (max(first[i]["cg_iters"], 1) * p.N * p.D))
            mu, s_, a = firsts[i]
            rel = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))  # noqa: E731
            parity[f"problem_{i}_D{p.D}"] = {"cg_iters": first[i]["cg_iters"], "relerr_mu": rel(mu, e.mu),
                                             "relerr_s": rel(s_, e.s), "relerr_alpha": rel(a, a_ref)}
        c = float(np.mean(per_elem_iter))
        em_time = sum(c * p.N * p.D * cg[:, i].mean() for i, p in enumerate(probs))
        cpu = {"value": round(1.0 / em_time, 6), "unit": "batch EM it/s", "cores": int(threads), "kind": "oracle",
               "sample": f"first E-step + M-step of problems {sample} (D = {[sizes[i] for i in sample]}) took "
                         f"{t_el:.1f}s on the host at the GPU's CG counts; the cost per (N*D element, CG "
                         f"iteration) scaled to all {n} problems at the GPU run's mean CG counts"}
        log(f"cpu oracle: {cpu['value']:.5f} batch EM it/s; parity {parity}")

    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "batch EM it/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32", "data": "synthetic",
        "config": {"workload": "batched_64", "problems": n, "D_min": min(sizes), "D_max": max(sizes),
                   "sum_ND": int(sum(p.N * p.D for p in probs)), "K": p0.K, "beta": p0.beta, "cg_tol": p0.tol,
                   "cg_max_iter": p0.max_iter, "T_em": T_em,
                   "form": "bf16 dictionaries (the problem), float32 CG, fp64 mean column; grouped launches "
                           "replayed from one captured graph",
                   "autotuner": plan, "cg_iters_per_em_mean": round(float(cg.mean()), 2)},
        "roofline": roofline, "cpu_baseline": cpu, "parity": parity,
    }
    print(json.dumps(out), flush=True)
    g.close()

def dct_bytes(p, which):
    """Bytes one launch of the DCT operator must move in a fused CG iteration
    (K float probe columns in P = ceil(K/2) complex pairs, the float64 mean
    column alone): rows in reads p, r, q, x and writes x, r, p, then writes
    the complex intermediate; the middle launch reads and writes the
    intermediate and reads the mask; rows out reads the intermediate, p, r
    and alpha and writes q."""
    K, D = p.K, p.D
    P = (K + 1) // 2
    inter = 8 * P + 16
    if which == "pass1":
        return D * (28 * K + 56 + inter)
    if which == "pass2":
        return D * (2 * inter + 8)
    return D * (inter + 12 * K + 44)


def run_dct(args):
    """The DCT dictionary (Sec. 4): inverse DCT of a length-D coefficient
    vector followed by N = D/4 observed samples.  A step is T_em EM
    iterations from alpha = 1.  Forms: the warm-started Jacobi-preconditioned
    float32 CG (`control`, the default: the previous iterate as the start,
    M^-1 = 1/(beta ||Phi e_k||^2 + alpha_k)) and plain float32 CG (`fp32`, the
    paper's solver), each with a float64 mean column.  Also reported for both:
    the time to a 2% NRMSE against the ground truth (the paper's
    high-dimensional DCT protocol), from the library's own per-EM-iteration
    event times."""
    import numpy as np
    import torch

    from paper_2202_12808_amd import synth
    from paper_2202_12808_amd.cofem import CoFEM

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    p = synth.WORKLOADS[args.workload](0)
    if args.tasks > 1:
        # the same dictionary law, beta, K and tolerance with T tasks sharing
        # alpha (a shared support, independent values per task)
        p = synth.dct_multitask(p.D, args.tasks, rho=float(np.count_nonzero(p.z)) / p.D, beta=p.beta, K=p.K,
                                tol=p.tol, max_iter=p.max_iter, T_em=p.T_em, seed=0,
                                name=f"{p.name}_tasks{args.tasks}")
    T_em = args.em_iters or p.T_em
    log(f"workload {p.name}: N={p.N} D={p.D} K={p.K} tasks={p.tasks} beta={p.beta} tol={p.tol} U={p.max_iter} "
        f"T_em={T_em} nnz={int(np.count_nonzero(p.z)) // p.tasks} "
        f"(inputs generated in {time.perf_counter() - t_gen:.1f}s)")
    if args.form is None:
        args.form = "control"
    if args.form not in ("fp32", "control"):
        print(f"--form {args.form} is not built for the DCT dictionary", file=sys.stderr, flush=True)
        sys.exit(2)
    rows = torch.from_numpy(p.rows.astype(np.int32)).to(dev)
    y = torch.from_numpy(p.y).to(dev)

    def make(form):
        ctl = form == "control"
        return CoFEM.dct(rows, y, p.D, p.beta, p.K, tol=p.tol, max_iter=p.max_iter, seed=p.seed, jacobi=ctl,
                         warm_start=ctl)

    g = make(args.form)
    ones = torch.ones(p.D, dtype=torch.float32, device=dev)
    calibration_copies(args, dev)

    def one_step(c):
        c.set_alpha(ones)
        c.set_iteration(1)
        return c.em_step(T_em)

    nz = np.linalg.norm(p.z)

    def estimate(c):
        # every task's mean (T x D), or the one mean (D)
        if p.tasks > 1:
            return c.means().cpu().numpy()
        return c.posterior()[0].cpu().numpy().astype(np.float64)

    def time_to_target(c, target=0.02):
        # one EM iteration at a time from alpha = 1, summing the library's
        # per-iteration event times (host NRMSE not counted)
        c.set_alpha(ones)
        c.set_iteration(1)
        t_ms, trace, reached = 0.0, [], None
        for it in range(2 * T_em):
            st = c.em_step(1)[0]
            t_ms += st["ms"]
            e = float(np.linalg.norm(estimate(c) - p.z) / nz)
            trace.append(round(e, 5))
            if e <= target:
                reached = {"em_iters": it + 1, "ms": round(t_ms, 3)}
                break
        return {"target_nrmse": target, "reached": reached, "nrmse_per_em_iter": trace}

    # the parity and CPU sample: the first EM iteration from alpha = 1 of the
    # plain form (the oracle's CG), on a context of its own
    gp = make("fp32")
    first = gp.em_step(1)[0]
    mu1, s1, a1 = [x.cpu().numpy().astype(np.float64) for x in gp.posterior()]
    if p.tasks > 1:
        mu1 = gp.means().cpu().numpy().T
    gp.close()
    for w in range(args.warmup):
        st = one_step(g)
        log(f"warmup {w + 1}/{args.warmup}: cg iters {sum(x['cg_iters'] for x in st)}")
    g.set_kernel_timing(0 if args.no_kernel_timing else args.timing_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        stats = one_step(g)
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cg_counts = [x["cg_iters"] for x in stats]
    mean_cg = float(np.mean(cg_counts))
    value = args.steps * T_em / elapsed
    nrmse = float(np.linalg.norm(estimate(g) - p.z) / nz)
    log(f"{value:.3f} EM it/s; CG iterations per EM iteration: mean {mean_cg:.1f}, min {min(cg_counts)}, "
        f"max {max(cg_counts)}; NRMSE vs ground truth {nrmse:.4f}")

    names = KERNEL_NAMES["dct"]
    if not args.no_kernel_timing:
        kt = g.kernel_timing()
        g.set_kernel_timing(False)
        total = {k: kt[k][0] for k in names}
        per = {k: kt[k][0] / max(kt[k][1], 1) for k in names}
        launches = {k: kt[k][1] for k in names}
        source = (f"HIP events around the launches of every {args.timing_every}-th CG iteration "
                  "during the timed steps")
    else:
        ms = g.time_operator(args.timing_reps)
        per = {k: ms[i] for i, k in enumerate(("pass1", "pass2", "update"))}
        total, launches = dict(per), {k: args.timing_reps for k in per}
        source = "cofem_time_operator back-to-back launches"
    dom = max(per, key=lambda k: total[k])
    nbytes = dct_bytes(p, dom)
    gbs = nbytes / (per[dom] * 1e-3) / 1e9
    traffic = stored_traffic("dct", names[dom], p.name)
    roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": names[dom],
                "bytes_per_launch": nbytes, "ms_per_launch": round(per[dom], 5), "timing": source,
                "kernels": {names[k]: {"ms_per_launch": round(per[k], 5), "launches": launches[k],
                                       "bytes_per_launch": dct_bytes(p, k),
                                       "gbs": round(dct_bytes(p, k) / (per[k] * 1e-3) / 1e9, 1)} for k in per}}
    log("per-launch us " + ", ".join(f"{names[k]} {per[k] * 1e3:.1f} "
                                    f"({dct_bytes(p, k) / (per[k] * 1e-3) / 1e9:.0f} GB/s)" for k in per))

    forms = {args.form: {"value": round(value, 4), "cg_iters_per_em": cg_counts, "nrmse_vs_truth": round(nrmse, 6),
                         "time_to_nrmse": time_to_target(g)}}
    log(f"form {args.form}: time to NRMSE 0.02 {forms[args.form]['time_to_nrmse']['reached']}")
    if not args.no_compare:
        other = "fp32" if args.form == "control" else "control"
        g2 = make(other)
        one_step(g2)  # warm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st2 = one_step(g2)
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t1
        forms[other] = {"value": round(T_em / el2, 4), "cg_iters_per_em": [x["cg_iters"] for x in st2],
                        "nrmse_vs_truth": round(float(np.linalg.norm(estimate(g2) - p.z) / nz), 6),
                        "time_to_nrmse": time_to_target(g2)}
        log(f"form {other}: {forms[other]['value']:.3f} EM it/s; CG per EM {forms[other]['cg_iters_per_em']}; "
            f"NRMSE {forms[other]['nrmse_vs_truth']}; time to NRMSE 0.02 {forms[other]['time_to_nrmse']['reached']}")
        g2.close()

    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle as O
        try:
            from threadpoolctl import threadpool_info
            threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [os.cpu_count()])
        except Exception:
            threads = os.cpu_count()
        from oracle import multitask as OM
        op = O.DctMaskOperator(p.rows, p.D)
        n1 = first["cg_iters"]
        tc0 = time.perf_counter()
        b0 = p.beta * op.apply_t(np.asarray(p.y, np.float64).reshape(p.tasks, p.N).T)
        e = OM.cofem_estep_mt(op, b0, p.beta, np.ones(p.D), p.K, p.tol, p.max_iter, p.seed, 1, fixed_iters=n1)
        a_ref, _ = OM.mstep_mt(e.mu, e.s)
        if p.tasks == 1:
            e.mu = e.mu[:, 0]
        t_sample = time.perf_counter() - tc0
        # the first E-step converges in very few iterations; time a few more
        # operator applications for a stable cost per CG iteration
        A = O.cofem_oracle.make_apply_A(op, p.beta, np.ones(p.D))
        V = np.ones((p.D, p.K + p.tasks))
        reps = 10
        tc1 = time.perf_counter()
        for _ in range(reps):
            A(V)
        per_cg = (time.perf_counter() - tc1) / reps
        cpu = {"value": round(1.0 / (per_cg * mean_cg), 5), "unit": "EM it/s", "cores": int(threads),
               "kind": "oracle",
               "sample": f"first E-step + M-step of {p.name} ({n1} CG iterations) took {t_sample:.2f}s on the "
                         f"host; {reps} operator applications on all {p.K + p.tasks} columns took {per_cg * 1e3:.1f} ms "
                         f"each; scaled to this form's mean of {mean_cg:.1f} CG iterations per EM iteration"}

        def rel(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))
        parity = {"step": 1, "cg_iters": n1, "relerr_mu": rel(mu1, e.mu), "relerr_s": rel(s1, e.s),
                  "relerr_alpha": rel(a1, a_ref), "nmse_mu": rel(mu1, e.mu) ** 2}
        log(f"cpu oracle: {cpu['value']:.4f} EM it/s on {threads} threads; parity {parity}")

    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "EM it/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": p.name, "N": p.N, "D": p.D, "K": p.K, "tasks": p.tasks, "beta": p.beta,
                   "cg_tol": p.tol, "cg_max_iter": p.max_iter, "T_em": T_em, "form": FORMS_DCT[args.form],
                   "cg_iters_per_em_mean": round(mean_cg, 2), "nrmse_vs_truth": round(nrmse, 6)},
        "roofline": roofline, "cpu_baseline": cpu, "parity": parity, "forms": forms,
    }
    print(json.dumps(out), flush=True)
    g.close()


def cpu_info():
    """Host CPU model and the number of cores this process may use."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([t.get("num_threads", 1) for t in threadpool_info()] or [os.cpu_count()])
    except Exception:
        return os.cpu_count()


def nmse(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.sum((a - ref) ** 2) / np.sum(ref ** 2))


CONV_FORM_ORDER = ("learned", "control", "fp32")


def run_conv(args):
    """The convolution dictionary (the metric's workload at 1024 x 1024, 9x9
    taps).  A step is T_em EM iterations from alpha = 1 (cofem_restart).  The
    headline form is the learned start; the non-learned control (previous
    iterate + Jacobi) and plain float32 CG are timed the same way and
    reported under "forms".  Every form's mean after the first m EM
    iterations is compared with the float64 oracle run of the control's
    algorithm over the same m iterations (its FFT route); that oracle run is
    also the CPU sample."""
    import torch

    from paper_2202_12808_amd import synth
    from paper_2202_12808_amd.cofem import CoFEM

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    p = synth.WORKLOADS[args.workload](0)
    T_em = args.em_iters or p.T_em
    m_ref = args.oracle_em_iters
    log(f"workload {p.name}: N={p.N} D={p.D} K={p.K} beta={p.beta} tol={p.tol} U={p.max_iter} T_em={T_em} "
        f"(inputs generated in {time.perf_counter() - t_gen:.1f}s)")
    form = args.form or "learned"
    if form not in CONV_FORM_ORDER:
        print(f"--form {form} is not built for the convolution dictionary", file=sys.stderr, flush=True)
        sys.exit(2)
    taps = torch.from_numpy(p.taps).to(dev)
    y = torch.from_numpy(p.y).to(dev)
    net = train_info = None
    if form == "learned" or not args.no_compare:
        net, train_info = train_predictor(p, dev, spectral=not args.no_spectral)

    def make(f):
        ctl = f == "control"
        spec = f in ("control", "learned") and not args.no_spectral
        c = CoFEM.conv(taps, y, p.H, p.W, p.beta, p.K, tol=p.tol, max_iter=p.max_iter, seed=p.seed, jacobi=ctl,
                       warm_start=ctl, spectral_start=spec)
        if f == "learned":
            c.set_predictor(net)
        return c

    calibration_copies(args, dev)

    def timed(f, kernel_timing):
        g = make(f)
        for _ in range(args.warmup):
            g.restart()
            g.em_step(T_em)
        if kernel_timing:
            g.set_kernel_timing(args.timing_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            g.restart()
            st = g.em_step(T_em)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res = {"value": args.steps * T_em / el, "elapsed": el, "stats": st,
               "mu_T": g.solution()[1].cpu().numpy()}
        if kernel_timing:
            res["kt"] = g.kernel_timing()
            res["kt_names"] = {"pass1": g.kernel_name("pass1"), "pass2": g.kernel_name("pass2")}
            g.set_kernel_timing(0)
        if not args.no_cpu_baseline:  # the first m EM iterations, for the float64 reference
            g.restart()
            res["stats_m"] = g.em_step(m_ref)
            res["mu_m"] = g.solution()[1].cpu().numpy()
        g.close()
        cg = [x["cg_iters"] for x in st]
        log(f"form {f}: {res['value']:.3f} EM it/s over {args.steps} steps of {T_em} EM iterations; "
            f"CG per EM {cg}")
        return res

    runs = {form: timed(form, not args.no_kernel_timing)}
    if not args.no_compare:
        for f in CONV_FORM_ORDER:
            if f != form:
                runs[f] = timed(f, False)
    head = runs[form]
    value, elapsed = head["value"], head["elapsed"]
    cg_counts = [x["cg_iters"] for x in head["stats"]]

    # roofline of the fused stencil iteration (the dominant kernel: the
    # persistent k_conv_ws at this size, or the per-tile k_conv_fused)
    roofline = None
    if "kt" in head:
        kname = head["kt_names"]["pass1"]
        kt = head["kt"]["pass1"]  # the fused iterations (a solve's first pass is timed apart, in "pass2")
        ms = kt[0] / max(kt[1], 1)
        nbytes = algorithmic_bytes(p, "pass1")
        nflops = algorithmic_flops(p, "pass1")
        gbs = nbytes / (ms * 1e-3) / 1e9
        tfs = nflops / (ms * 1e-3) / 1e12
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "traffic": stored_traffic("conv_ws" if kname == "k_conv_ws" else "conv", kname, p.name),
                    "kernel": kname,
                    "bytes_per_launch": nbytes, "ms_per_launch": round(ms, 5), "launches": kt[1],
                    "timing": f"HIP events around the launches of every {args.timing_every}-th CG iteration "
                              "during the timed steps",
                    "alu": {"flops_per_launch": nflops, "achieved_tflops": round(tfs, 2),
                            "peak_issue_tflops": FP32_VALU_ISSUE_TFS, "frac_issue": round(tfs / FP32_VALU_ISSUE_TFS, 4),
                            "peak_published_tflops": FP32_VALU_PEAK_TFS,
                            "frac_published": round(tfs / FP32_VALU_PEAK_TFS, 4)}}
        k0 = head["kt"]["pass2"]
        if k0[1]:
            roofline["first_pass"] = {"kernel": head["kt_names"]["pass2"], "ms_per_launch": round(k0[0] / k0[1], 5),
                                      "launches": k0[1]}
        log(f"roofline: {kname} {ms * 1e3:.1f} us/launch, {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f}% of "
            f"HBM), {tfs:.2f} TFLOP/s ({100 * tfs / FP32_VALU_ISSUE_TFS:.1f}% of the non-packed fp32 issue rate)")

    # the float64 reference: the oracle run of the control's algorithm over
    # the first m EM iterations (FFT route), also the CPU sample
    traj = cpu = None
    nz = np.linalg.norm(p.z)
    forms = {}
    for f, r in runs.items():
        forms[f] = {"value": round(r["value"], 4), "cg_iters_per_em": [x["cg_iters"] for x in r["stats"]],
                    "nrmse_vs_truth": round(float(np.linalg.norm(r["mu_T"] - p.z) / nz), 6)}
    if "fp32" in runs:
        ref = runs["fp32"]["mu_T"]
        forms["nmse_mu_T_vs_fp32"] = {f: nmse(r["mu_T"], ref) for f, r in runs.items()}
    if train_info is not None:
        forms["training"] = train_info
    if not args.no_cpu_baseline:
        import oracle as O
        model, ncpu = cpu_info()
        op = O.ConvOperatorFFT(p.taps.astype(np.float64), p.H, p.W)
        y64 = p.y.astype(np.float64)
        log(f"oracle reference: {m_ref} EM iterations of the control's algorithm on {op.workers} threads ...")
        t0 = time.perf_counter()
        ref = O.cofem(op, y64, p.beta, m_ref, p.K, tol=p.tol, max_iter=p.max_iter, seed=p.seed, warm_start=True,
                      jacobi=True, spectral_start=not args.no_spectral)
        el = time.perf_counter() - t0
        cg_or = [x["cg_iters"] for x in ref.stats]
        # the per-EM-iteration work besides CG (probes, diagonal estimate, M-step)
        t1 = time.perf_counter()
        Pm = O.rademacher_probes(p.seed, 1, p.K, p.D)
        O.mstep(ref.mu, O.diag_estimate(Pm, Pm))
        c_em = time.perf_counter() - t1
        c_cg = max(el - m_ref * c_em, 1e-9) / max(sum(cg_or), 1)
        # one thread: two CG iterations of the first E-step
        try:
            from threadpoolctl import threadpool_limits
        except Exception:
            threadpool_limits = None
        op1 = O.ConvOperatorFFT(p.taps.astype(np.float64), p.H, p.W)
        op1.workers = 1
        b0 = p.beta * op1.apply_t(y64)
        ctx = threadpool_limits(1) if threadpool_limits else None
        t2 = time.perf_counter()
        if ctx:
            with ctx:
                O.cofem_estep(op1, b0, p.beta, np.ones(p.D), p.K, p.tol, p.max_iter, p.seed, 1, fixed_iters=2)
        else:
            O.cofem_estep(op1, b0, p.beta, np.ones(p.D), p.K, p.tol, p.max_iter, p.seed, 1, fixed_iters=2)
        el1 = time.perf_counter() - t2
        c_cg1 = max(el1 - c_em, 1e-9) / 2.0

        def em_rate(per_cg, per_em):
            return T_em / sum(per_cg * c + per_em for c in cg_counts)

        cpu = {"value": round(em_rate(c_cg, c_em), 6), "unit": "EM it/s", "cores": int(op.workers), "kind": "oracle",
               "sample": f"float64 oracle ({op.workers} FFT workers, {blas_threads()} BLAS threads) ran the first "
                         f"{m_ref} EM iterations of the control's algorithm ({sum(cg_or)} CG iterations, "
                         f"{cg_or}) in {el:.1f}s: {c_cg * 1e3:.0f} ms per CG iteration plus {c_em * 1e3:.0f} ms "
                         f"per EM iteration (probes, diagonal estimate, M-step); scaled to the headline run's "
                         f"{sum(cg_counts)} CG iterations over {T_em} EM iterations",
               "first_m_em_per_s": round(m_ref / el, 6),
               "one_thread": {"value": round(em_rate(c_cg1, c_em), 6), "ms_per_cg_iter": round(c_cg1 * 1e3, 1),
                              "sample": "two CG iterations of the first E-step on one thread, scaled the same way"},
               "host": {"cpu_model": model, "nproc": ncpu}}
        traj = {"em_iters": m_ref, "reference": "float64 oracle, control's algorithm (warm start + Jacobi"
                                                + ("" if args.no_spectral else ", exact first E-step") + "), FFT route", "oracle_cg_iters": cg_or, "host_seconds": round(el, 1),
                "nmse_mu_vs_oracle": {f: nmse(r["mu_m"], ref.mu) for f, r in runs.items()},
                "cg_iters_gpu": {f: [x["cg_iters"] for x in r["stats_m"]] for f, r in runs.items()}}
        log(f"cpu oracle: {cpu['value']:.5f} EM it/s ({c_cg * 1e3:.0f} ms per CG iteration on {op.workers} threads, "
            f"{c_cg1 * 1e3:.0f} ms on one); NMSE of mu after {m_ref} EM iterations vs the oracle "
            f"{traj['nmse_mu_vs_oracle']}")

    secondary = time_to_target = None
    if not args.no_secondary:
        a2 = argparse.Namespace(**vars(args))
        a2.workload, a2.form, a2.em_iters = "dense_4096x16384", None, 0
        if net is not None:
            net.close()
        torch.cuda.empty_cache()
        secondary = run_dense(a2, emit=False)
        torch.cuda.empty_cache()
        time_to_target = dct_time_to_target()

    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "EM it/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": p.name, "N": p.N, "D": p.D, "K": p.K, "beta": p.beta, "cg_tol": p.tol,
                   "cg_max_iter": p.max_iter, "T_em": T_em, "form": form,
                   "form_detail": FORMS[form] + ("" if args.no_spectral or form == "fp32" else SPECTRAL_NOTE),
                   "cg_iters_per_em_mean": round(float(np.mean(cg_counts)), 2),
                   "nrmse_vs_truth": forms[form]["nrmse_vs_truth"]},
        "roofline": roofline, "cpu_baseline": cpu, "forms": forms, "oracle_trajectory": traj,
        "secondary": secondary, "time_to_target": time_to_target,
    }
    print(json.dumps(out), flush=True)


def dct_time_to_target(em_tol=1e-3, target=0.02):
    """The high-dimensional DCT protocol of Sec. 4.2 (Fig. 1(f)): from alpha =
    1, the EM iterations and the library's own per-iteration event time until
    the mean reaches an NRMSE of 2% against the ground truth, for the
    warm-started Jacobi form at D = 2^18; and where the EM-level stop rule
    (cofem_em_run: relative change of 1/alpha below em_tol) ends the same run."""
    import torch

    from paper_2202_12808_amd import synth
    from paper_2202_12808_amd.cofem import CoFEM

    p = synth.dct_262144(0)
    rows = torch.from_numpy(p.rows.astype(np.int32)).cuda()
    y = torch.from_numpy(p.y).cuda()
    nz = np.linalg.norm(p.z)
    out = {"workload": p.name, "form": "control", "target_nrmse": target}
    with CoFEM.dct(rows, y, p.D, p.beta, p.K, tol=p.tol, max_iter=p.max_iter, seed=p.seed, jacobi=True,
                   warm_start=True) as g:
        g.em_step(5)  # warm the kernels
        g.restart()
        t_ms, reached, trace = 0.0, None, []
        for it in range(2 * p.T_em):
            st = g.em_step(1)[0]
            t_ms += st["ms"]
            e = float(np.linalg.norm(g.posterior()[0].cpu().numpy().astype(np.float64) - p.z) / nz)
            trace.append(round(e, 5))
            if e <= target:
                reached = {"em_iters": it + 1, "ms": round(t_ms, 3)}
                break
        out["reached"] = reached
        out["nrmse_per_em_iter"] = trace
        g.restart()
        st = g.em_run(2 * p.T_em, em_tol)
        out["em_stop"] = {"em_tol": em_tol, "em_iters": len(st), "ms": round(sum(x["ms"] for x in st), 3),
                          "nrmse": round(float(np.linalg.norm(g.posterior()[0].cpu().numpy().astype(np.float64)
                                                              - p.z) / nz), 6),
                          "gamma_change_last": st[-1]["gamma_change"]}
    log(f"time to NRMSE {target} on {p.name}: {out['reached']}; EM stop at {out['em_stop']}")
    return out


def run_dense(args, emit=True):
    """Dense workloads.  The headline form is the mixed-precision one
    (bf16 dictionary in the inner CG solves, iterative refinement on the
    float32 dictionary's true residual, each E-step started from the previous
    mean and diagonal estimate); plain float32 CG started the same way
    (fp32_warm) and from zero (fp32) are timed on the same inputs."""
    import torch

    from paper_2202_12808_amd import synth
    from paper_2202_12808_amd.cofem import CoFEM

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    p = synth.WORKLOADS[args.workload](0)
    T_em = args.em_iters or p.T_em
    log(f"workload {p.name}: N={p.N} D={p.D} K={p.K} beta={p.beta} tol={p.tol} U={p.max_iter} "
        f"T_em={T_em} (inputs generated in {time.perf_counter() - t_gen:.1f}s)")
    form = args.form or "bf16_ir"
    if form not in DENSE_FORM_ORDER:
        print(f"--form {form} is not built for dense dictionaries", file=sys.stderr, flush=True)
        sys.exit(2)
    y = torch.from_numpy(p.y).to(dev)
    phi = torch.from_numpy(p.phi).to(dev)
    calibration_copies(args, dev)

    def make(f):
        prec = "bf16_ir" if f == "bf16_ir" else "fp32"
        warm = (f == "bf16_ir" and not args.no_warm) or f == "fp32_warm"
        # the warm-started forms also take the Jacobi diagonal; plain fp32 stays plain CG
        return CoFEM.dense(phi, y, p.beta, p.K, tol=p.tol, max_iter=p.max_iter, seed=p.seed, precision=prec,
                           ir_inner_tol=args.ir_inner_tol, warm_start=warm, jacobi=warm and not args.no_jacobi)

    def timed(f, kernel_timing):
        g = make(f)
        for _ in range(max(args.warmup, 1)):
            g.restart()
            g.em_step(T_em)
        if kernel_timing:
            g.set_kernel_timing(args.timing_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            g.restart()
            st = g.em_step(T_em)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res = {"value": args.steps * T_em / el, "elapsed": el, "stats": st,
               "mu_T": g.solution()[1].cpu().numpy()}
        if kernel_timing:
            res["kt"] = g.kernel_timing()
            g.set_kernel_timing(0)
        # the first E-step alone (parity and the CPU sample)
        g.restart()
        res["first"] = g.em_step(1)[0]
        res["first_post"] = [x.cpu().numpy().astype(np.float64) for x in g.posterior()]
        res["first_sweeps"] = g.ir_sweeps() if f == "bf16_ir" else None
        g.close()
        cg = [x["cg_iters"] for x in st]
        log(f"form {f}: {res['value']:.3f} EM it/s; CG per EM mean {np.mean(cg):.1f}")
        return res

    runs = {form: timed(form, not args.no_kernel_timing)}
    if not args.no_compare:
        for f in DENSE_FORM_ORDER:
            if f != form:
                runs[f] = timed(f, False)
    head = runs[form]
    value, elapsed = head["value"], head["elapsed"]
    cg_counts = [x["cg_iters"] for x in head["stats"]]
    mean_cg = float(np.mean(cg_counts))
    nz = np.linalg.norm(p.z)

    roofline = None
    if "kt" in head:
        names = KERNEL_NAMES["dense_bf16_ir" if form == "bf16_ir" else "dense"]
        kt = head["kt"]
        per = {k: kt[k][0] / max(kt[k][1], 1) for k in names}
        dom = max(("pass1", "pass2"), key=lambda k: kt[k][0])
        phi_bytes = 2 if form == "bf16_ir" else 4
        nbytes = algorithmic_bytes(p, dom, phi_bytes)
        gbs = nbytes / (per[dom] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "traffic": stored_traffic("dense_bf16_ir" if form == "bf16_ir" else "dense", names[dom], p.name),
                    "kernel": names[dom], "bytes_per_launch": nbytes, "ms_per_launch": round(per[dom], 5),
                    "timing": f"HIP events around the launches of every {args.timing_every}-th CG iteration "
                              "during the timed steps",
                    "kernels": {names[k]: {"ms_per_launch": round(per[k], 5), "launches": kt[k][1]} for k in names}}
        log(f"roofline: {names[dom]} {per[dom] * 1e3:.1f} us/launch, {gbs:.0f} GB/s "
            f"({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM)")

    forms = {f: {"value": round(r["value"], 4), "cg_iters_per_em_mean": round(float(np.mean(
        [x["cg_iters"] for x in r["stats"]])), 2), "nrmse_vs_truth": round(float(np.linalg.norm(r["mu_T"] - p.z) / nz), 6)}
        for f, r in runs.items()}
    if "bf16_ir" in runs:
        forms["bf16_ir"]["ir_sweeps_per_em_mean"] = round(float(np.mean([x["ir_sweeps"] for x in
                                                                         runs["bf16_ir"]["stats"]])), 2)
    if "fp32" in runs:
        forms["nmse_mu_T_vs_fp32"] = {f: nmse(r["mu_T"], runs["fp32"]["mu_T"]) for f, r in runs.items()}

    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle as O
        threads = blas_threads()
        op = O.DenseOperator(p.phi.astype(np.float64))
        first = head["first"]
        n1 = first["cg_iters"]
        tc0 = time.perf_counter()
        b0 = p.beta * op.apply_t(p.y.astype(np.float64))
        if form == "bf16_ir":
            opb = O.DenseOperator(synth.round_to_bf16(p.phi).astype(np.float64))
            e, _ = O.cofem_estep_ir(op, opb, b0, p.beta, np.ones(p.D), p.K, p.tol, args.ir_inner_tol or 0.1,
                                    p.max_iter, 20, p.seed, 1, fixed_inner=head["first_sweeps"])
            # inner iterations plus the outer residuals: one operator application each
            n_ops = n1 + len(head["first_sweeps"])
        else:
            e = O.cofem_estep(op, b0, p.beta, np.ones(p.D), p.K, p.tol, p.max_iter, p.seed, 1, fixed_iters=n1)
            n_ops = n1
        a_ref, _ = O.mstep(e.mu, e.s)
        t_sample = time.perf_counter() - tc0
        per_cg = t_sample / max(n_ops, 1)
        scale = float(np.mean([x["cg_iters"] for x in runs["fp32"]["stats"]])) if "fp32" in runs else mean_cg
        model, ncpu = cpu_info()
        cpu = {"value": round(1.0 / (per_cg * scale), 5), "unit": "EM it/s", "cores": int(threads), "kind": "oracle",
               "sample": f"first E-step + M-step of {p.name} ({n_ops} operator applications) took {t_sample:.2f}s "
                         f"on the host; scaled to the plain float32 form's mean of {scale:.1f} CG iterations per "
                         f"EM iteration", "host": {"cpu_model": model, "nproc": ncpu}}
        mu1, s1, a1 = head["first_post"]
        parity = {"step": 1, "cg_iters": n1, "relerr_mu": float(np.linalg.norm(mu1 - e.mu) / np.linalg.norm(e.mu)),
                  "relerr_s": float(np.linalg.norm(s1 - e.s) / np.linalg.norm(e.s)),
                  "relerr_inv_alpha": float(np.linalg.norm(1 / a1 - 1 / a_ref) / np.linalg.norm(1 / a_ref))}
        if head["first_sweeps"] is not None:
            parity["ir_sweeps"] = head["first_sweeps"]
        log(f"cpu oracle: {cpu['value']:.4f} EM it/s on {threads} threads; parity {parity}")

    out = {
        "metric": METRIC if emit else "EM it/s of the dense workload (secondary)", "value": round(value, 4),
        "unit": "EM it/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16+f32" if form == "bf16_ir" else "f32", "data": "synthetic",
        "config": {"workload": p.name, "N": p.N, "D": p.D, "K": p.K, "beta": p.beta, "cg_tol": p.tol,
                   "cg_max_iter": p.max_iter, "T_em": T_em, "form": form, "form_detail": FORMS[form],
                   "cg_iters_per_em_mean": round(mean_cg, 2), "nrmse_vs_truth": forms[form]["nrmse_vs_truth"]},
        "roofline": roofline, "cpu_baseline": cpu, "parity": parity, "forms": forms,
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="conv_1024x1024_k9",
                    choices=["conv_1024x1024_k9", "conv_256x256_k7", "dense_4096x16384", "dense_256x1024",
                             "batched_64", "dct_4096", "dct_262144"])
    ap.add_argument("--em-iters", type=int, default=0, help="EM iterations per step (default: workload's)")
    ap.add_argument("--tasks", type=int, default=1,
                    help="DCT workloads: T > 1 tasks sharing alpha (multi-task SBL)")
    ap.add_argument("--timing-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the float64 oracle (CPU sample, parity and the NMSE reference)")
    ap.add_argument("--oracle-em-iters", type=int, default=5,
                    help="conv workloads: EM iterations of the float64 oracle reference and CPU sample")
    ap.add_argument("--timing-every", type=int, default=13,
                    help="time the launches of every n-th CG iteration with HIP events (1: all; each timed "
                         "iteration's events cost a few microseconds of stream time; 13 is coprime to the "
                         "solver's 8-iteration polling chunks, so the timed iterations fall evenly on every "
                         "chunk position)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time the steps without the per-launch events (roofline from cofem_time_operator)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="first run 3 plain device copies of this many MiB (counter calibration)")
    ap.add_argument("--form", default=None, choices=sorted(FORMS),
                    help="solver form timed for the headline value (default: learned for conv, bf16_ir for "
                         "dense, control for DCT)")
    ap.add_argument("--no-warm", action="store_true",
                    help="bf16_ir: start every E-step's refinement from zero instead of the previous mean and "
                         "diagonal estimate")
    ap.add_argument("--ir-inner-tol", type=float, default=0.0,
                    help="bf16_ir: relative tolerance of each inner solve (0: the library default, 0.1)")
    ap.add_argument("--no-compare", action="store_true",
                    help="time only the headline form")
    ap.add_argument("--no-secondary", action="store_true",
                    help="conv workloads: skip the dense 4096 x 16384 summary carried in the same line")
    ap.add_argument("--no-jacobi", action="store_true",
                    help="dense workloads: run the warm-started forms without the Jacobi diagonal")
    ap.add_argument("--no-spectral", action="store_true",
                    help="conv workloads: start the control and learned forms' first E-step from zero instead "
                         "of the 2D-DFT solve")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr, flush=True)
        sys.exit(2)

    if args.workload == "batched_64":
        return run_batched(args)
    if args.workload.startswith("dct"):
        return run_dct(args)
    if args.workload.startswith("conv"):
        return run_conv(args)
    return run_dense(args)


if __name__ == "__main__":
    main()
