#!/usr/bin/env python3
"""Benchmark of the borehole FWI hot path on one MI355X.

A step is one full preconditioned gradient-descent FWI iteration over the
workload, every stage in the HIP library: moduli (Eq. 3-4), then per group
of shots the autograd-wrapped forward with checkpoints (Eq. 2) -- traces out
of the BoreholeFWI torch.autograd.Function, the misfit of Eq. 1 as a torch
expression, loss.backward() running the checkpoint recompute, the adjoint
with the fused correlation (Eq. 6-8) and the finalize -- then the diagonal
preconditioner, the update (Eq. 9-10) and the velocities (Eq. 11-12).
Inputs are seeded synthetic models already resident in HBM.

Default workload (c3): 64 tool positions every 0.15 m over one layered
formation, each shot 256 x 4096 cells of 2.5 mm plus a 20-cell PML, 8000
steps of 0.25 us, 10 kHz Ricker, 13 receivers, checkpoints every 250 steps
with sequential recompute; the loss is summed over shots.

Prints one JSON line.  value = Gcell-updates/s of the whole iteration
(2 x cell-steps per iteration / wall time: one forward and one adjoint sweep).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Gcell-updates/s fwd+adj+grad and % HBM roofline; "
          "shots·FWI-iters/s batched vs plain")
HBM_PEAK_GBS = 8000.0
# vector issue peak without packed FP32: one wave64 VALU instruction per CU
# and clock, 256 CUs at 2.4 GHz
VALU_PEAK_GIPS = 256 * 2.4
FP32_VECTOR_PEAK_TFLOPS = 157.3
# Algorithmic bytes per cell and step (FP32) of the unblocked step kernels:
# the forward reads and writes 6 fields and reads lambda, mu, rho; the
# recompute also stores v_r, v_z; the adjoint with the fused correlation reads
# and writes 6 adjoint fields, reads lambda, mu, rho and the stored v_r, v_z,
# and reads and writes g_lambda, g_mu and the illumination.
FWD_BYTES_PER_CELL_STEP = 60
REC_BYTES_PER_CELL_STEP = 68
ADJ_BYTES_PER_CELL_STEP = 92
# The same adjoint run as T-step blocks with the state in registers: per cell
# and block the 6 adjoint fields, the model and the 3 accumulators cross HBM
# once (48 + 12 + 24 B), the stored velocities once per step (8 B per step).
ADJ_BLOCK_BYTES_PER_CELL = 84
ADJ_BLOCK_BYTES_PER_CELL_STEP = 8
# each extra output (the density correlation, the pseudo-Hessian) reads and
# writes two more accumulator planes per cell and launch
ADJ_BLOCK_BYTES_PER_CELL_X = 16

# HBM traffic of the adjoint time block, from rocprofv3 --pmc runs of
#   bench.py --workload W --nt 250 --steps 1 --warmup 0 --no-cpu-baseline
#            --plain-shots 0 --no-kernel-times
# restricted to the adjoint kernels: DRAM read and write requests of the L2
# (TCC_EA0_RDREQ_DRAM_32B, TCC_EA0_WRREQ_WRITE_DRAM_32B, in 32-byte units;
# a device copy of 1 GiB reads 1.000 GiB and writes 1.000 GiB on them,
# profiles/copy_calibration.md), the mean per dispatch summed over the
# interior and PML kernels of one block.  An entry holds only for the kernel
# sources it was measured on (SHA-256 of PMC_SOURCES: the adjoint block kernel
# and the device code it includes), the same shapes, tile map and workload;
# otherwise traffic is null.
PMC_SOURCES = ("paper_2005_00281_amd/csrc/bhfwi_tb_adj.hip",
               "paper_2005_00281_amd/csrc/bhfwi_tb_fwd.hip",
               "paper_2005_00281_amd/csrc/bhfwi_kernels.hip",
               "paper_2005_00281_amd/csrc/bhfwi_internal.h")
PMC_TRAFFIC = {
    # (kernel, tile_map, workload, sources sha256[:16]): (read bytes, write bytes)
    ("k_adj_tb<6, 32, 16, 0, 0> + k_adj_tb<6, 32, 16, 1, 0>", 1, "c3", "f361bc00e3e764f0"):
        (8127040826, 3470398762),
}

# Vector instructions of the same adjoint block, from a rocprofv3 --pmc run
# of the same command with SQ_INSTS_VALU (wave64 instructions, summed over the
# interior and PML kernels of one block, mean per dispatch); the same keys.
PMC_VALU = {
    ("k_adj_tb<6, 32, 16, 0, 0> + k_adj_tb<6, 32, 16, 1, 0>", 1, "c3", "f361bc00e3e764f0"):
        1202725870,
}

# temporally blocked shapes (T, tile rows incl. halo, waves) of both kernels,
# and those of the forward kernel only
TB_SHAPES = [(2, 16, 4), (3, 16, 4), (4, 16, 4), (2, 16, 8), (3, 16, 8), (4, 16, 8),
             (2, 24, 8), (3, 24, 8), (4, 24, 8), (6, 24, 8), (4, 32, 8), (6, 32, 8),
             (8, 32, 8), (2, 16, 16), (3, 16, 16), (4, 16, 16), (4, 32, 16), (6, 32, 16),
             (8, 32, 16)]
FWD_ONLY_SHAPES = [(4, 48, 16), (6, 48, 16), (8, 48, 16), (4, 64, 16), (8, 64, 16)]
ADJ_ONLY_SHAPES = [(4, 48, 16), (6, 48, 16), (8, 48, 16), (8, 64, 16)]
# workloads whose configuration stores the whole velocity history (the
# others checkpoint every ckpt steps and recompute)
FULL_HISTORY_WORKLOADS = ("c1",)


def adj_shape(tune):
    """(T, rows, waves) of the adjoint kernel under a tune (T < 2: one step
    per launch)."""
    if tune["adj_tb_steps"] >= 2:
        return (tune["adj_tb_steps"], tune["adj_tb_rows"], tune["adj_tb_waves"])
    if tune["adj_tb_steps"] == 1:
        return (0, 0, 0)
    return (tune["tb_steps"], tune["tb_rows"], tune["tb_waves"])


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in PMC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def adjoint_blocks(nt_shots, nt_max, seg, T):
    """Adjoint launches each shot takes part in: steps run from nt_max - 1
    down, cut at the segment boundaries j*seg, T steps per launch within a
    segment; a shot takes part while the block's lowest step is below its
    own nt."""
    out = [0] * len(nt_shots)
    for j0 in range(0, nt_max, seg):
        n = min(j0 + seg, nt_max) - 1
        while n >= j0:
            nb = min(T, n - j0 + 1)
            lo = n - nb + 1
            for s, nt in enumerate(nt_shots):
                if lo < nt:
                    out[s] += 1
            n -= nb
    return out


def copy_bandwidth():
    """Device-to-device copy of 2 GiB (reads + writes counted): the practical
    HBM ceiling on this GPU, best of 5."""
    import torch
    n = 1 << 29
    src = torch.ones(n, device="cuda")
    dst = torch.empty(n, device="cuda")
    dst.copy_(src)
    best = 1e30
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * 4 * n / (best * 1e-3) / 1e9


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def host_cpu():
    """(model name, logical CPUs this process may run on)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(w, nt_sample, max_workers):
    """The FP64 oracle, as it is, on the host cores: one worker thread per
    shot (the oracle's C calls release the interpreter lock), each running
    the first nt_sample steps of its own shot -- forward modelling of the
    start model, misfit and the checkpointed gradient evaluation -- after an
    untimed forward of the true model for its observed data.  Rate per
    cell-step of the gradient evaluation, summed over the shots, over the
    wall time of the parallel part."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import oracle
    model, ncpu = host_cpu()
    workers = max(1, min(max_workers, ncpu, len(w.shots)))
    shots = list(range(workers))

    def setup(s):
        sh = w.shots[s]
        g = oracle.Geom(sh.nr, sh.nz, sh.pr, sh.pz, sh.dr, sh.dz, sh.dt, min(nt_sample, sh.nt),
                        sh.f0, sh.vmax, sh.src_k, sh.rec_k)
        win = lambda a: np.ascontiguousarray(w.window(a, s))  # noqa: E731
        rho = win(w.rho)
        lt, mt = oracle.moduli(win(w.vp_true), win(w.vs_true), rho)
        lam, mu = oracle.moduli(win(w.vp_start), win(w.vs_start), rho)
        dobs = oracle.forward(g, lt, mt, rho, sh.wavelet)
        return g, lam, mu, rho, sh.wavelet, dobs

    def run(args):
        g, lam, mu, rho, wav, dobs = args
        d = oracle.forward(g, lam, mu, rho, wav)
        _, r = oracle.misfit(d, dobs)
        oracle.gradient(g, lam, mu, rho, wav, r, seg=50)
        return g.NR * g.NZ * g.nt

    with ThreadPoolExecutor(workers) as ex:
        prepared = list(ex.map(setup, shots))
        t0 = time.perf_counter()
        cs = sum(ex.map(run, prepared))
        dt = time.perf_counter() - t0
    return {"value": round(2 * cs / dt / 1e9, 5), "unit": "Gcell-updates/s", "cores": workers,
            "kind": "oracle",
            "sample": "%d shot(s) of %s in parallel (one host thread each), the first %d of "
                      "%d steps of each (%.3g cell-steps in all): forward + misfit + "
                      "checkpointed gradient, %.1f s wall" % (
                          workers, w.name, min(nt_sample, w.shots[0].nt), w.shots[0].nt, cs, dt),
            "host": {"cpu_model": model, "logical_cpus": ncpu}}


def semblance_bench(steps):
    """Starting-model stage at the 128-shot workload's scale: the slowness-time
    coherence of 128 gathers of 13 receivers x 16000 samples (0.25 us; a P
    and a weaker S plane arrival, Vp/Vs in [1.6, 1.9], in noise), 560
    slownesses of 1 us/m from 150 us/m, 150 us windows every 10 samples, and
    the P and S picks.  Work model per (gather, slowness, staged sample): 13
    interpolated reads at 5 FP32 operations each (shift split, two loads
    folded into one FMA, stack add, energy FMA) plus the square of the stack;
    per window two double differences.  Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2005_00281_amd as P
    dev = torch.device("cuda", 0)
    G, M, nt, dt = 128, 13, 16000, 0.25e-6
    p0, dp, npp, stride, win = 150e-6, 1e-6, 560, 10, 600
    ntau = (nt - win) // stride + 1
    rng = np.random.default_rng(11)
    t = np.arange(nt) * dt
    off = 0.1524 * np.arange(M)
    x = np.empty((G, M, nt), np.float32)
    true_p, true_s = np.empty(G), np.empty(G)
    for g in range(G):
        vp = rng.uniform(3000, 5500)
        sp, ss = 1 / vp, rng.uniform(1.6, 1.9) / vp
        true_p[g], true_s[g] = sp, ss
        for m in range(M):
            a = (np.pi * 8e3 * (t - 1e-3 - sp * off[m])) ** 2
            b = (np.pi * 8e3 * (t - 2e-3 - ss * off[m])) ** 2
            x[g, m] = (3 * (1 - 2 * a) * np.exp(-a) + (1 - 2 * b) * np.exp(-b) +
                       0.05 * rng.standard_normal(nt))
    xt = torch.as_tensor(x, device=dev)
    ot = torch.as_tensor(np.tile(off, (G, 1)), dtype=torch.float32, device=dev)
    P.semblance(xt, dt, ot, p0, dp, npp, stride, ntau, win, energy=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        coh, en = P.semblance(xt, dt, ot, p0, dp, npp, stride, ntau, win, energy=True)
        pP, _ = P.semblance_pick(coh, p0, dp, 1 / 6000, 1 / 2000, energy=en, rel_floor=1e-6)
        pS, _ = P.semblance_pick(coh, p0, dp, 0.0, 0.999 / 1500, p_ref=pP, ref_scale=1.4,
                                 energy=en, rel_floor=1e-6)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    span = 2048
    chunk = (span - win) // stride + 1
    staged = G * npp * sum(min(span, (min(ntau, c + chunk) - 1 - c) * stride + win)
                           for c in range(0, ntau, chunk))
    flops = staged * (5 * M + 1)
    achieved = flops / (ms * 1e-3) / 1e12
    out = {"metric": "starting-model semblance: coherence cells per second", "unit": "Gcells/s",
           "value": round(G * npp * ntau / (ms * 1e-3) / 1e9, 3), "ms_per_step": round(ms, 3),
           "steps": steps, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "128 gathers x 13 receivers x 16000 samples, 560 slownesses, "
                                  "%d windows of %d samples" % (ntau, win)},
           "max_pick_error_us_per_m": round(1e6 * max(
               np.abs(pP.cpu().numpy() - true_p).max(), np.abs(pS.cpu().numpy() - true_s).max()), 3),
           "roofline": {"bound": "alu", "achieved": round(achieved, 2),
                        "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None}}
    print(json.dumps(out), flush=True)


def copy_calibration():
    """One device copy of 1 GiB from memory that is not in any cache, for
    scaling the L2-to-memory counters (bytes known exactly)."""
    import torch
    n = 1 << 28  # floats
    src = torch.ones(n, device="cuda")
    dst = torch.empty(n, device="cuda")
    evict = torch.empty(1 << 28, device="cuda")
    evict.fill_(2.0)  # pushes src out of L2 and the infinity cache
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "copy_kib": 4 * n / 1024}))


def trace_gaps(path):
    """Idle time between the kernels of a rocprofv3 kernel trace (its
    kernel_trace.csv): dispatches sorted by start, the gap after each one up
    to the next start (0 when they overlap), summed over the whole trace and
    over consecutive pairs of time-step kernels (the launch gaps a persistent
    launch would remove; gaps of 1 ms or more between them are host-side
    pauses and are counted apart).  Prints one JSON line."""
    import csv
    ev = []
    with open(path) as f:
        for r in csv.DictReader(f):
            ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    ev.sort()
    step = ("k_fwd_tb", "k_adj_tb", "k_fwd_step", "k_adj_step", "k_fwd4", "k_adj4")
    is_step = [any(x in name for x in step) for _, _, name in ev]
    busy, end_max, gaps, step_gaps = 0, None, [], []
    for j, (t0, t1, _) in enumerate(ev):
        if end_max is None or t0 >= end_max:
            busy += t1 - t0
            if end_max is not None:
                gaps.append(t0 - end_max)
                if is_step[j] and is_step[j - 1]:
                    step_gaps.append(t0 - end_max)
        elif t1 > end_max:
            busy += t1 - end_max
        end_max = t1 if end_max is None else max(end_max, t1)
    span = ev[-1][1] - ev[0][0] if ev else 0
    # gaps of a millisecond or more are host-side pauses (stage boundaries,
    # synchronisations), not launch latency
    pauses = [g for g in step_gaps if g >= 1000000]
    step_gaps = [g for g in step_gaps if g < 1000000]
    sg = sorted(step_gaps)
    step_busy = sum(t1 - t0 for (t0, t1, _), s in zip(ev, is_step) if s)
    out = {"trace": os.path.basename(path), "dispatches": len(ev),
           "step_dispatches": sum(is_step), "span_ms": round(span / 1e6, 3),
           "busy_ms": round(busy / 1e6, 3), "idle_ms": round(sum(gaps) / 1e6, 3),
           "step_kernel_ms": round(step_busy / 1e6, 3),
           "step_pairs": len(sg) + len(pauses), "step_gap_ms": round(sum(sg) / 1e6, 3),
           "host_pauses": len(pauses), "host_pause_ms": round(sum(pauses) / 1e6, 3),
           "step_gap_frac_of_step_time": round(sum(sg) / step_busy, 5) if step_busy else None,
           "step_gap_us": {"mean": round(sum(sg) / len(sg) / 1e3, 3) if sg else None,
                           "p50": round(sg[len(sg) // 2] / 1e3, 3) if sg else None,
                           "p99": round(sg[int(0.99 * (len(sg) - 1))] / 1e3, 3) if sg else None,
                           "max": round(sg[-1] / 1e3, 3) if sg else None}}
    print(json.dumps(out), flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--nt", type=int, default=0,
                    help="record length override (profiling runs: the kernels and tune of the "
                         "full-length workload on a shorter record)")
    ap.add_argument("--direct", action="store_true",
                    help="drive the C-ABI directly (Inversion without the autograd op)")
    ap.add_argument("--rows", type=int, default=0, help="rows per wave (0: library default)")
    ap.add_argument("--tb", type=int, default=-1,
                    help="forward steps per launch in the LDS-tiled kernels (-1: default)")
    ap.add_argument("--tb-rows", type=int, default=0)
    ap.add_argument("--tb-waves", type=int, default=0)
    ap.add_argument("--tile-map", type=int, default=-1)
    ap.add_argument("--adj-tb", type=int, default=-1,
                    help="adjoint steps per launch (0: as the forward, 1: one per launch)")
    ap.add_argument("--pml-overlap", type=int, default=-1)
    ap.add_argument("--full-history", type=int, default=None,
                    help="1: keep the velocity history of every step (no checkpoints, no "
                         "recompute); 0: checkpoints and recompute; -1: full history when the "
                         "plan is one group that fits the budget with it; default: as the "
                         "workload's configuration states")
    ap.add_argument("--fwd-overlap", type=int, default=-1,
                    help="tune fwd_tile_overlap (-1: as tuned)")
    ap.add_argument("--rec-overlap", type=int, default=-1,
                    help="1: recompute segment j-1 on a second stream during the adjoint of "
                         "segment j (default: the tune's)")
    ap.add_argument("--adj-tb-rows", type=int, default=0)
    ap.add_argument("--adj-tb-waves", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2005_00281_amd",
                                                         "tune_cache.json"),
                    help="autotuner results per device and survey shape ('' : none)")
    ap.add_argument("--retune", action="store_true",
                    help="re-run the autotuner and record its choice in the tune cache")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=300)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="most host threads for the oracle baseline (one shot each)")
    ap.add_argument("--plain-shots", type=int, default=2,
                    help="shots timed in the plain one-shot, one-step-per-launch form")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="HBM budget for the planner (0: 80%% of the device)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--trace-gaps", default="",
                    help="summarise the idle gaps of a rocprofv3 kernel_trace.csv and exit")
    ap.add_argument("--semblance", action="store_true",
                    help="measure the starting-model semblance stage instead")
    ap.add_argument("--progress", action="store_true",
                    help="synchronise and log after every shot group (long workloads)")
    ap.add_argument("--no-kernel-times", action="store_true",
                    help="skip the event-timed gradient evaluation (no roofline)")
    ap.add_argument("--kt-groups", type=int, default=0,
                    help="shot groups in the per-kernel timing pass (0: all)")
    ap.add_argument("--line-search", type=int, default=-1,
                    help="1: parabolic line search each iteration (one extra forward); "
                         "-1: as the workload specifies (the 128-shot workload uses it)")
    ap.add_argument("--order", type=int, default=2, choices=(2, 4),
                    help="spatial order of the step (4: the four-point stencils, one step "
                         "per launch)")
    ap.add_argument("--density", action="store_true",
                    help="joint inversion: the density gradient and step as well (an "
                         "extension; the paper keeps the density fixed)")
    ap.add_argument("--precond", default="illum", choices=("illum", "pseudo_hessian"),
                    help="diagonal of the preconditioner")
    ap.add_argument("--taper", default="",
                    help="r0,r1 in metres: a radial taper on top of the diagonal")
    ap.add_argument("--sweep", action="store_true",
                    help="time one gradient evaluation per temporally blocked shape "
                         "(stderr only) before the benchmark")
    return ap.parse_args()


def main():
    args = parse()
    if args.trace_gaps:
        trace_gaps(args.trace_gaps)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.semblance:
        semblance_bench(max(1, args.steps))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    import paper_2005_00281_amd as P
    from paper_2005_00281_amd.fwi import Inversion
    from paper_2005_00281_amd import plan as planner

    dev = torch.device("cuda", 0)
    nt_key = None
    if args.nt:  # the kernels are those tuned for the full-length record
        import inspect
        par = inspect.signature(workloads.CONFIGS.get(args.workload, workloads.tiny)).parameters
        if "nt" not in par:
            sys.exit("--nt: workload %s has no single record length" % args.workload)
        nt_key = par["nt"].default
    w = workloads.make(args.workload, **({"nt": args.nt} if args.nt else {}))
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)  # noqa: E731
    log("workload", args.workload, "shots", len(w.shots), "grid", w.shots[0].NR, w.shots[0].NZ,
        "nt", w.shots[0].nt)
    budget = (args.budget_gb * 1e9 if args.budget_gb > 0
              else 0.8 * torch.cuda.get_device_properties(0).total_memory)
    autograd = not args.direct
    if autograd and args.precond != "illum":
        log("--precond %s: the pseudo-Hessian diagonal needs the direct path" % args.precond)
        autograd = False
    pl = planner.plan(w.shots, budget, ckpt_every=w.meta.get("ckpt"))
    log("plan: %d group(s) of %s shots, checkpoint every %s steps, %.1f GB workspaces" % (
        len(pl.groups), [len(g) for g in pl.groups], pl.ckpt_every, pl.bytes_workspace / 1e9))
    rho = f32(w.rho)
    surveys, wavs = [], []
    for g, K in zip(pl.groups, pl.ckpt_every):
        sv = P.Survey([w.shots[s] for s in g], (w.NRg, w.NZg), ckpt_every=K, order=args.order)
        surveys.append(sv)
        wavs.append(sv.pack_wavelets([w.shots[s].wavelet for s in g]))
    lam_t, mu_t = P.moduli(f32(w.vp_true), f32(w.vs_true), rho)
    observed = []
    for g, (sv, wav) in enumerate(zip(surveys, wavs)):
        observed.append(sv.fwd_model(lam_t, mu_t, rho, wav).clone())
        sv.free_workspaces()
        if args.progress:
            torch.cuda.synchronize()
            log("observed data: group %d of %d" % (g + 1, len(surveys)))
    del lam_t, mu_t
    mask = torch.as_tensor(w.mask, device=dev)
    line_search = (bool(w.meta.get("line_search", False)) if args.line_search < 0
                   else bool(args.line_search))
    if args.density and line_search:
        log("--density: the line search steps lambda and mu only; running without it")
        line_search = False
    row_weight = None
    if args.taper:
        r0, r1 = (float(x) for x in args.taper.split(","))
        row_weight = P.radial_taper(w.NRg, w.shots[0].dr, r0, r1)
        if autograd:
            log("--taper: the row weights need the direct path")
            autograd = False
    if args.tb >= 0 or args.adj_tb >= 0 or args.rows or args.no_autotune:
        for sv in surveys:
            sv.set_tune(rows_per_wave=args.rows or None,
                        tb_steps=args.tb if args.tb >= 0 else None,
                        tb_rows=args.tb_rows or None, tb_waves=args.tb_waves or None,
                        tile_map=args.tile_map if args.tile_map >= 0 else None,
                        adj_tb_steps=args.adj_tb if args.adj_tb >= 0 else None,
                        adj_tb_rows=args.adj_tb_rows or None,
                        adj_tb_waves=args.adj_tb_waves or None)
    else:
        # the autotuner's choice for this device and survey shape: from the
        # tune cache when it holds one (--retune re-measures and records it)
        lam_s, mu_s = P.moduli(f32(w.vp_start), f32(w.vs_start), rho)
        cache = args.tune_cache or None
        if cache and args.retune and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            for sv in surveys:
                table.pop(sv.shape_key(nt_key), None)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        t_at = time.perf_counter()
        tuned = {}  # set of shot shapes -> tune of the first group that has it
        for g, (sv, wav) in enumerate(zip(surveys, wavs)):
            shapes = frozenset((sh.nr, sh.nz, sh.pr, sh.pz, sh.nt)
                               for sh in (w.shots[s] for s in pl.groups[g]))
            if shapes in tuned:  # a group of the same shot shapes: same kernels
                sv.set_tune(**tuned[shapes])
                continue
            entry = sv.autotune(lam_s, mu_s, rho, wav, cache=cache, key=sv.shape_key(nt_key))
            tuned[shapes] = entry["tune"]
            log("tune key %s%s" % (sv.shape_key(nt_key)[:60],
                                   " (cached)" if entry.get("cached") else ""))
        log("autotune %.1f s -> %s%s" % (time.perf_counter() - t_at, entry["tune"],
                                          " (tune cache)" if entry.get("cached") else ""))
        del lam_s, mu_s
    if args.rec_overlap >= 0:
        for sv in surveys:
            sv.set_tune(rec_overlap=args.rec_overlap)
    if args.fwd_overlap >= 0:
        for sv in surveys:
            sv.set_tune(fwd_tile_overlap=args.fwd_overlap)
    fh = args.full_history
    if fh is None:
        fh = 1 if args.workload in FULL_HISTORY_WORKLOADS else 0
    if fh < 0:
        full = len(surveys) == 1 and surveys[0].use_full_history_if_fits(budget)
        if not full:
            for sv in surveys:
                sv.set_tune(full_history=0)
    else:
        for sv in surveys:
            sv.set_tune(full_history=fh)
        full = bool(fh)
    log("velocity history: %s (%.1f GB per group)" % (
        "every step" if full else "checkpoints", surveys[0].device_bytes() / 1e9))
    # the shared workspaces of the iteration are sized for the tune in force
    inv = Inversion(surveys, f32(w.vp_start), f32(w.vs_start), rho, wavs, observed, mask,
                    line_search=line_search, density=args.density, precond=args.precond,
                    row_weight=row_weight, autograd=autograd)
    if args.progress:
        def _progress(stage, g):
            torch.cuda.synchronize()
            log("%s: group %d of %d done" % (stage, g + 1, len(surveys)))
        inv.after_group = _progress
    if args.sweep:
        sweep(inv, surveys)
    if args.no_graph:
        for sv in surveys:
            sv.set_tune(use_graph=0)
    if args.pml_overlap >= 0:
        for sv in surveys:
            sv.set_tune(pml_overlap=args.pml_overlap)
    sv = surveys[0]
    tune = sv.get_tune()
    cell_steps = sum(x.sizes.cell_steps for x in surveys)

    for _ in range(args.warmup):
        inv.iterate()
    torch.cuda.synchronize()
    log("warmup done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Js = []
    for _ in range(args.steps):
        J, a = inv.iterate()
        Js.append(J)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / max(1, args.steps)
    value = 2 * cell_steps / (ms * 1e-3) / 1e9
    log("ms/iteration %.2f, J %s" % (ms, [round(float(j), 6) for j in Js]))

    roofline, kernels = kernel_roofline(args, inv, surveys, tune, full)

    # iteration-level figure: the algorithmic bytes of the unblocked path per
    # cell-step (forward, recompute, adjoint; without the recompute when the
    # whole history is kept; plus a forward for the line search) over the
    # iteration time; temporal blocking moves far fewer bytes, so this is an
    # effective bandwidth and can exceed 1
    it_bytes = (FWD_BYTES_PER_CELL_STEP + ADJ_BYTES_PER_CELL_STEP +
                (8 if full else REC_BYTES_PER_CELL_STEP) +
                (FWD_BYTES_PER_CELL_STEP if line_search else 0))
    it_frac = (it_bytes * cell_steps / (ms * 1e-3)) / (HBM_PEAK_GBS * 1e9)

    plain = None
    if args.plain_shots > 0:
        del inv
        torch.cuda.empty_cache()
        plain = plain_form(args, w, pl, observed, mask, rho, line_search, row_weight, autograd,
                           full, f32)

    copy_bw = copy_bandwidth()
    log("device copy %.1f GB/s" % copy_bw)

    base = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        base = cpu_baseline(w, args.cpu_sample_steps, args.cpu_workers)

    history = ("velocity history of every step (no checkpoints, no recompute)" if full else
               "checkpoints every %s steps, %s recompute" % (
                   pl.ckpt_every, "overlapped" if tune["rec_overlap"] else "sequential"))
    sh0 = w.shots[0]
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%s: %d shot(s), %dx%d padded cells (shot 0), %d steps "
                               "(shot 0), dt %.3g s, f0 %.3g Hz, %d receivers; %s; %s" % (
                                   args.workload, len(w.shots), sh0.NR, sh0.NZ, sh0.nt, sh0.dt,
                                   sh0.f0, len(sh0.rec_k), history,
                                   "autograd op + loss.backward()" if autograd
                                   else "C-ABI driven directly"),
                   "history": "full" if full else "checkpoints",
                   "autograd": autograd,
                   "cell_steps_per_iteration": int(cell_steps),
                   "line_search": line_search,
                   "order": args.order,
                   "density": bool(args.density), "precond": args.precond,
                   "taper": args.taper or None,
                   "kernel_shapes": sv.kernel_shapes(),
                   "tune": tune},
        "roofline": roofline,
        "iteration_effective_frac": round(it_frac, 4),
        "iteration_bytes_per_cell_step": it_bytes,
        "copy_GBs": round(copy_bw, 1),
        "shots_iters_per_s": round(len(w.shots) / (ms * 1e-3), 4),
        "plain": plain,
        "batched_vs_plain": (round(len(w.shots) / (ms * 1e-3) / plain["shots_iters_per_s"], 3)
                             if plain else None),
        "plan": {"groups": [len(g) for g in pl.groups], "ckpt_every": pl.ckpt_every,
                 "workspace_gb": round(pl.bytes_workspace / 1e9, 2)},
        "kernels": kernels,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


def kernel_roofline(args, inv, surveys, tune, full):
    """Per-kernel durations from one more (untimed) gradient evaluation of the
    first --kt-groups shot groups (all by default), every time-step launch
    bracketed by HIP events on the stream it runs on; the roofline of the
    adjoint block (the largest share of GPU time) from them."""
    if args.no_kernel_times:
        return None, {}
    timed = surveys[:args.kt_groups] if args.kt_groups > 0 else surveys
    kt = {"fwd": [0.0, 0], "rec": [0.0, 0], "adj": [0.0, 0]}
    for x in timed:
        x.set_tune(use_graph=0, time_kernels=1)
        x.kernel_times(reset=True)
    all_surveys, inv.surveys = inv.surveys, timed
    inv.gradient()
    inv.surveys = all_surveys
    for x in timed:
        for k, (ms_, n_) in x.kernel_times(reset=True).items():
            kt[k][0] += ms_
            kt[k][1] += n_
        x.set_tune(use_graph=tune["use_graph"], time_kernels=0)
    cs_timed = sum(x.sizes.cell_steps for x in timed)
    per_cs = {"fwd": FWD_BYTES_PER_CELL_STEP, "rec": REC_BYTES_PER_CELL_STEP,
              "adj": ADJ_BYTES_PER_CELL_STEP}
    kernels = {}
    for k, (kms, kn) in kt.items():
        if kn:
            kernels[k] = {"avg_us": round(kms * 1e3 / kn, 3), "launches": kn,
                          "effective_GBs": round(per_cs[k] * cs_timed / (kms * 1e-3) / 1e9, 1)}
    adj_ms, adj_n = kt["adj"]
    if not adj_n:
        return None, kernels
    sv = surveys[0]
    kshapes = sv.kernel_shapes()
    xm = (1 if args.density else 0) | (2 if args.precond == "pseudo_hessian" else 0)
    ka, kp = (kshapes["adj_x"], kshapes["adj_x_pml"]) if xm else (kshapes["adj"],
                                                                  kshapes["adj_pml"])
    b4 = sv.order4_blocks
    T = (ka[0] if (args.order == 2 and ka[0] >= 2) else
         b4[0] if (args.order == 4 and b4[0] >= 2) else 1)
    kname = (("k_adj4_tb<%d, %d, %d, 0, %d> + k_adj4_tb<%d, %d, %d, 1, %d>" % (
              b4 + (xm,) + b4 + (xm,)) if b4[0] >= 2 else "k_adj4<%d>" % xm) if args.order == 4
             else "k_adj_tb<%d, %d, %d, 0, %d> + k_adj_tb<%d, %d, %d, 1, %d>" % (
             ka + (xm,) + kp + (xm,))
             if ka[0] >= 2
             else "k_adj_step<%d>" % (tune["rows_per_wave"] if tune["rows_per_wave"] <= 4 else 0))
    adj_avg_s = adj_ms * 1e-3 / adj_n
    # algorithmic bytes of the blocked adjoint over the timed groups: per cell
    # and launch the state, model and accumulators, per cell and step the
    # stored velocities
    per_cell = ADJ_BLOCK_BYTES_PER_CELL + ADJ_BLOCK_BYTES_PER_CELL_X * bin(xm).count("1")
    floor = 0
    for x in timed:
        nts = [sh.nt for sh in x.shots]
        seg = max(nts) if full else x.sizes.ckpt_every
        blocks = adjoint_blocks(nts, max(nts), seg, T)
        for sh, nb in zip(x.shots, blocks):
            floor += sh.cells * (per_cell * nb +
                                 ADJ_BLOCK_BYTES_PER_CELL_STEP * sh.nt)
    floor_per_launch = floor / adj_n
    floor_GBs = floor_per_launch / adj_avg_s / 1e9
    eff_GBs = ADJ_BYTES_PER_CELL_STEP * cs_timed / adj_n / adj_avg_s / 1e9
    pmc_key = (kname, tune.get("tile_map", 1), args.workload, kernel_sources_sha())
    pmc = PMC_TRAFFIC.get(pmc_key)
    traffic = None if pmc is None else int(pmc[0] + pmc[1])
    traffic_GBs = None if traffic is None else traffic / adj_avg_s / 1e9
    if traffic is not None:
        achieved, basis = traffic_GBs, ("rocprofv3 DRAM read + write requests of the L2 per "
                                         "launch (profiles/), over the HIP-event launch time")
    else:
        achieved, basis = floor_GBs, ("algorithmic bytes of the blocked adjoint per launch "
                                      "(counters not taken for these kernel sources)")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "traffic_unit": "bytes per launch",
                "basis": basis,
                "kernel": kname, "avg_launch_us": round(adj_avg_s * 1e6, 3),
                "launches": adj_n, "steps_per_launch": round(
                    sum(x.sizes.nt_max for x in timed) / adj_n, 3),
                "floor_bytes_per_launch": int(floor_per_launch),
                "floor_GBs": round(floor_GBs, 1),
                "floor_frac": round(floor_GBs / HBM_PEAK_GBS, 4),
                "floor_model": "%d B per cell and launch + %d B per cell and step" % (
                    per_cell, ADJ_BLOCK_BYTES_PER_CELL_STEP),
                "effective_GBs": round(eff_GBs, 1),
                "effective_frac": round(eff_GBs / HBM_PEAK_GBS, 4),
                "effective_model": "%d B per cell-step, unblocked" % ADJ_BYTES_PER_CELL_STEP}
    valu = PMC_VALU.get(pmc_key)
    if valu is not None:  # the resource that bounds these kernels: vector issue
        gips = valu / adj_avg_s / 1e9
        roofline["valu"] = {"bound": "alu", "achieved": round(gips, 1),
                            "peak": VALU_PEAK_GIPS, "unit": "G wave64 VALU instructions/s",
                            "frac": round(gips / VALU_PEAK_GIPS, 4),
                            "instructions_per_launch": valu,
                            "basis": "rocprofv3 SQ_INSTS_VALU per launch (profiles/), over "
                                     "the HIP-event launch time"}
    return roofline, kernels


def plain_form(args, w, pl, observed, mask, rho, line_search, row_weight, autograd, full, f32):
    """The plain form: one shot per survey, one step per launch, no graph; the
    same checkpoint interval and history mode, the same iteration (autograd
    op, line search) as the batched run.  Per-shot iteration times,
    extrapolated over all shots by cell-steps."""
    import torch
    import paper_2005_00281_amd as P
    from paper_2005_00281_amd.fwi import Inversion
    per_cs = []
    for s_ in range(min(args.plain_shots, len(w.shots))):
        sh = w.shots[s_]
        g_ = [i for i, g in enumerate(pl.groups) if s_ in g][0]
        sv1 = P.Survey([sh], (w.NRg, w.NZg), ckpt_every=pl.ckpt_every[g_], order=args.order)
        sv1.set_tune(rows_per_wave=2, tb_steps=0, adj_tb_steps=0, use_graph=0,
                     full_history=1 if full else 0)
        if args.order == 4:
            sv1.set_order4_blocks(0)
        wav1 = sv1.pack_wavelets([sh.wavelet])
        off = sum(len(w.shots[q].rec_k) * w.shots[q].nt for q in pl.groups[g_] if q < s_)
        obs1 = observed[g_][off: off + len(sh.rec_k) * sh.nt].clone()
        inv1 = Inversion(sv1, f32(w.vp_start), f32(w.vs_start), rho.clone(), wav1, obs1,
                         mask, line_search=line_search, density=args.density,
                         precond=args.precond, row_weight=row_weight, autograd=autograd)
        inv1.iterate()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inv1.iterate()
        torch.cuda.synchronize()
        per_cs.append((time.perf_counter() - t0) / (sh.cells * sh.nt))
        del inv1, sv1
        torch.cuda.empty_cache()
    rate = sum(per_cs) / len(per_cs)
    t_plain = rate * sum(sh.cells * sh.nt for sh in w.shots)
    return {"shots_iters_per_s": round(len(w.shots) / t_plain, 4),
            "ms_per_iteration": round(t_plain * 1e3, 1),
            "measured_shots": len(per_cs), "extrapolated": len(per_cs) < len(w.shots),
            "form": "one shot per launch sequence, one step per launch (wave march, 2 rows "
                    "per wave), no HIP graph; same checkpoint interval and history mode (%s), "
                    "same iteration (%s)" % ("full" if full else "checkpoints",
                                             "autograd op" if autograd else "direct C-ABI")}


def sweep(inv, surveys):
    """One gradient evaluation per temporally blocked shape (stderr only)."""
    import torch
    keep = surveys[0].get_tune()
    a0 = adj_shape(keep)

    def timed(**kw):
        for x in surveys:
            x.set_tune(**kw)
        inv.gradient()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inv.gradient()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3

    # forward shapes with the adjoint held at the tuned one, then the reverse
    for (T, R, W_) in TB_SHAPES + FWD_ONLY_SHAPES:
        for tmap in (0, 1):
            ms = timed(tb_steps=T, tb_rows=R, tb_waves=W_, tile_map=tmap,
                       adj_tb_steps=a0[0] if a0[0] >= 2 else 1, adj_tb_rows=a0[1],
                       adj_tb_waves=a0[2])
            log("sweep fwd T %d rows %d waves %d map %d: %.2f ms per gradient" % (
                T, R, W_, tmap, ms))
    for x in surveys:
        x.set_tune(**keep)
    for (T, R, W_) in TB_SHAPES + ADJ_ONLY_SHAPES:
        ms = timed(adj_tb_steps=T, adj_tb_rows=R, adj_tb_waves=W_)
        log("sweep adj T %d rows %d waves %d: %.2f ms per gradient" % (T, R, W_, ms))
    for x in surveys:
        x.set_tune(**keep)
    for ovl in (0, 1):
        # the PML stream and the recompute stream are not combined
        rov = 0 if ovl else keep["rec_overlap"]
        log("sweep pml_overlap %d (rec_overlap %d): %.2f ms per gradient" % (
            ovl, rov, timed(pml_overlap=ovl, rec_overlap=rov)))
    for x in surveys:
        x.set_tune(**keep)


if __name__ == "__main__":
    main()
