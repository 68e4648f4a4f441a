#!/usr/bin/env python3
"""Benchmark of the direct-summation force path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]

Headline workload: Newton all-pairs on a Plummer sphere of N = 262144
particles (scale radius 1, seed 102), equal masses 1/N, softening 0.01,
FP32, i-set = j-set.  One step is the whole path for one set of positions:
pgh_set_xmj (pack the j-particles into the library's records) followed by
pgh_calc_newton (accelerations and potentials), the GRAPE call sequence of
the paper's sample driver (Sec. 3.6).  Inputs are resident in device memory
before the timed region.

Prints ONE JSON line with the headline value (interactions per second), the
roofline object of the dominant kernel (pgh_calc_newton, FP32 ALU bound, 38
flops per interaction as the paper counts them, against the 157.3 TFLOP/s
FP32 vector peak), the FP64 oracle timed on a bounded sample on the host
cores, and secondary measurements of the other force paths.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

# 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 x 2.4 GHz: the factor 2 is packed FP32 or, as these
# kernels use it, the dual issue of two single FP32 instructions per quad-cycle
PEAK_FP32_TFLOPS = 157.3
NEWTON_FLOPS = 38  # per interaction, the paper's count (Sec. 5.1)
TABLE_FLOPS = 20  # per interaction, this project's count of the FP32 ops of the table loop


# Counters of the headline kernel per variant, from rocprofv3 --pmc runs of
# `bench.py --no-extras --no-cpu --variant NAME --copy-calibration 256`:
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch of k_newton_allpairs), each
# scaled by what the counter reads for a 256 MiB device-to-device copy, and
# SQ_INSTS_VALU_FLOPS_FP32 (x 64 per dispatch / interactions).  Valid only for
# the kernel sources they were taken on (their SHA-256); otherwise the bench
# reports them as null.
MEASURED = {
    "sources_sha256": "325486dddd3df0a060c6bcc4e60caff126f310cb2756c711cf358a22d6b7ad8d",
    # the 256 MiB copy: FETCH_SIZE 131091 KiB (x2.0), WRITE_SIZE 262144 KiB (x1.0)
    "fetch_factor": 2.0, "write_factor": 1.0,
    "by_variant": {
        # j split in 8 shares: 32 MiB of partial sums written, read back by k_combine_split
        "ki=4 jt=256 u=2": {"fetch_kib": 18319.9, "write_kib": 32768,
                            "valu_flops_per_interaction": 21.0},
        # j split in 2 shares
        "ki=1 jt=256 u=8": {"fetch_kib": 17944.1, "write_kib": 8192,
                            "valu_flops_per_interaction": 21.0},
        "ki=1 jt=64 u=8": {"fetch_kib": 17943.1, "write_kib": 8192,
                           "valu_flops_per_interaction": 21.1},
        # j split in 4 shares
        "ki=2 jt=256 u=4": {"fetch_kib": 17946.3, "write_kib": 16384,
                            "valu_flops_per_interaction": 21.0},
    },
}
KERNEL_SOURCES = ("paper_1203_4037_amd/csrc/newton.hip", "paper_1203_4037_amd/csrc/newton_pair.h",
                  "paper_1203_4037_amd/csrc/split.h")


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counters_for(variant_name, refine):
    """The recorded counters of this variant (no rsqrt refinement), or None
    when they were taken on other kernel sources or not at all."""
    t = MEASURED
    c = t["by_variant"].get(variant_name)
    if c is None or refine != 0 or t["sources_sha256"] != sources_sha256():
        return None
    return c


def measured_traffic(variant_name, refine):
    """HBM bytes per dispatch of the headline kernel, or None."""
    c = counters_for(variant_name, refine)
    if c is None:
        return None
    t = MEASURED
    return (c["fetch_kib"] * t["fetch_factor"] + c["write_kib"] * t["write_factor"]) * 1024.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the built-in default variant instead of the autotuned one")
    ap.add_argument("--variant", default=None, metavar="NAME",
                    help="time this all-pairs Newton variant instead of the autotuned one "
                         "(for profiling one variant)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target wall time of the CPU baseline sample")
    ap.add_argument("--replays", type=int, default=0,
                    help="graph replays per secondary measurement (0: the built-in counts; "
                         "profiler runs use a few)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (a known-size "
                         "reference for the HBM byte counters of a profiler run)")
    ap.add_argument("--only-extra", default=None, metavar="NAME",
                    help="run only the named secondary workload (e.g. tree_code) and print "
                         "its JSON; for profiling one workload")
    return ap.parse_args()


class KernelTimer:
    """HIP events around library calls on torch's current stream (the stream
    the library launches on)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = []

    def __enter__(self):
        self.a = self.torch.cuda.Event(enable_timing=True)
        self.b = self.torch.cuda.Event(enable_timing=True)
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self.pairs.append((self.a, self.b))

    def times_ms(self):
        self.torch.cuda.synchronize()
        return np.array([a.elapsed_time(b) for a, b in self.pairs])

    def mean_ms(self):
        return float(np.mean(self.times_ms()))


def time_steps(torch, step, steps, warmup):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cpu_baseline(x, y, z, m, eps, target_s, synth=None):
    """FP64 oracle (plain loops, OpenMP over i) on a sample of i-particles
    against all j, scaled to interactions per second; with synth, also the
    oracle's rate on the other configs (oracle_configs)."""
    import oracle
    configs = oracle_configs(synth) if synth is not None else None
    n = x.size
    e2 = np.float32(eps) ** 2
    cal = np.arange(0, n, max(1, n // 256))
    t0 = time.perf_counter()
    oracle.newton(x[cal], y[cal], z[cal], np.full(cal.size, e2, np.float32), x, y, z, m)
    rate = cal.size * n / (time.perf_counter() - t0)
    ns = int(min(n, max(256, rate * target_s / n)))
    idx = np.linspace(0, n - 1, ns).astype(np.int64)
    t0 = time.perf_counter()
    oracle.newton(x[idx], y[idx], z[idx], np.full(ns, e2, np.float32), x, y, z, m)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    one = one_core_rate(x, y, z, m, eps, rate / max(1, threads))
    return {"value": ns * n / dt, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, {ns} evenly spaced i-particles x all {n} j-particles "
                      f"({ns * n:.3e} interactions) in {dt:.1f} s",
            "value_1core": one, "cpu_model": cpu_model(), "configs": configs}


def oracle_configs(synth):
    """The FP64 oracle on every config with all host threads: config 1 full
    (Newton, N = 1024), config 3 full (table force on the 4^3-cell lists),
    config 4 on a stratified sample of 512 of its 16384 lists (the longest
    and the shortest by work, the rest evenly spaced in work order), config 5
    forward full (Newton all-pairs, N = 65536) and backward on a 4096-i
    slice.  Interactions per second each, with what was timed."""
    import oracle
    out = {}

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    n = 1024
    x, y, z = synth.plummer(n, 101)
    m = synth.equal_masses(n)
    e2 = np.full(n, np.float32(1.0 / 64) ** 2, np.float32)
    dt = timed(lambda: oracle.newton(x, y, z, e2, x, y, z, m))
    out["newton_allpairs_N1024"] = {"interactions_per_s": n * n / dt, "sample": "full"}
    n = 262144
    x, y, z = synth.uniform_box(n, 103)
    m = synth.equal_masses(n)
    s = synth.cell_grid_items(x, y, z, m, ncell=64, block=4)
    rcut, eps = 3.0 / 256, 1.0 / 1280
    tab = oracle.table_build(4, 6, float(np.float32(rcut)), oracle.SHAPE_S2PP, eps)
    dt = timed(lambda: oracle.lut_items(s.items, s.xi, s.yi, s.zi, s.xj, s.yj, s.zj, s.mj, 4, 6,
                                        float(np.float32(rcut)), tab))
    out["table_cell_lists_block4"] = {"interactions_per_s": s.interactions / dt, "sample": "full"}
    del s
    t = synth.tree_style_items(1 << 22, 16384, 104)
    cost = t.items[:, 1].astype(np.int64) * t.items[:, 3]
    order = np.argsort(cost)
    pick = order[np.unique(np.linspace(0, len(order) - 1, 512).round().astype(np.int64))]
    # the sampled lists' i-rows and j-ranges copied out compactly, so the
    # timed call widens only the sample to FP64
    it = t.items[pick].astype(np.int64)
    rows = np.concatenate([np.arange(a, a + b) for a, b in it[:, :2]])
    cols = np.concatenate([np.arange(a, a + b) for a, b in it[:, 2:]])
    ci = np.stack([np.concatenate([[0], np.cumsum(it[:, 1])[:-1]]), it[:, 1],
                   np.concatenate([[0], np.cumsum(it[:, 3])[:-1]]), it[:, 3]], 1)
    xi, yi, zi = t.xi[rows], t.yi[rows], t.zi[rows]
    xj, yj, zj, mj = t.xj[cols], t.yj[cols], t.zj[cols], t.mj[cols]
    e2 = np.full(rows.size, np.float32(1e-3) ** 2, np.float32)
    dt = timed(lambda: oracle.newton_items(ci, xi, yi, zi, e2, xj, yj, zj, mj))
    inter = float((it[:, 1] * it[:, 3]).sum())
    out["newton_batched_tree_lists"] = {"interactions_per_s": inter / dt,
                                        "sample": f"{len(pick)} of {len(t.items)} lists, {inter:.3e} interactions"}
    del t
    n = 65536
    x, y, z = synth.plummer(n, 105)
    m = synth.equal_masses(n)
    wx, wy, wz = synth.weights(n, 106)
    e2 = np.full(n, np.float32(0.01) ** 2, np.float32)
    dt = timed(lambda: oracle.newton(x, y, z, e2, x, y, z, m))
    out["adjoint_forward_N65536"] = {"interactions_per_s": float(n) * n / dt, "sample": "full"}
    k = 4096
    dt = timed(lambda: oracle.newton_bwd(x[:k], y[:k], z[:k], e2[:k], x, y, z, m,
                                         wx[:k], wy[:k], wz[:k]))
    out["adjoint_backward_N65536"] = {"interactions_per_s": float(k) * n / dt,
                                      "sample": f"{k} i-particles x {n} j-particles"}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def one_core_rate(x, y, z, m, eps, guess):
    """The oracle's rate on one thread (a child process with OMP_NUM_THREADS=1),
    on about 3 s of work; None when the child fails."""
    import subprocess
    import tempfile
    n = x.size
    ns = int(min(n, max(16, guess * 3.0 / n)))
    with tempfile.TemporaryDirectory() as d:
        np.savez(os.path.join(d, "in.npz"), x=x, y=y, z=z, m=m)
        code = ("import sys, time, numpy as np, oracle\n"
                f"a = np.load({os.path.join(d, 'in.npz')!r})\n"
                "x, y, z, m = a['x'], a['y'], a['z'], a['m']\n"
                f"ns, e2 = {ns}, np.float32({eps}) ** 2\n"
                "idx = np.linspace(0, x.size - 1, ns).astype(np.int64)\n"
                "t0 = time.perf_counter()\n"
                "oracle.newton(x[idx], y[idx], z[idx], np.full(ns, e2, np.float32), x, y, z, m)\n"
                "print(ns * x.size / (time.perf_counter() - t0))\n")
        env = dict(os.environ, OMP_NUM_THREADS="1",
                   PYTHONPATH=os.path.dirname(os.path.abspath(__file__)))
        try:
            out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                                 text=True, timeout=120)
            return float(out.stdout.strip().splitlines()[-1])
        except (subprocess.SubprocessError, ValueError, IndexError):
            return None


def newton_allpairs(torch, pgh, synth, args):
    n = args.n
    x, y, z = synth.plummer(n, 102)
    m = synth.equal_masses(n)
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    out = [torch.empty(n, device="cuda") for _ in range(4)]
    ctx = pgh.Context(0)
    ctx.set_eps_to_all(0.01)
    pgh.pgh_set_stream(ctx.h, torch.cuda.current_stream().cuda_stream)
    tuned = None
    if args.variant:
        fam = pgh.PGH_FAMILY_NEWTON_ALLPAIRS
        names = [pgh.pgh_variant_name(fam, v) for v in range(pgh.pgh_variant_count(fam))]
        if args.variant not in names:
            print(f"unknown variant {args.variant!r}; one of {names}", file=sys.stderr)
            sys.exit(2)
        ctx.set_variant(fam, names.index(args.variant))
    elif not args.no_tune:
        # the library's autotuner picks the tile shape on this very workload
        ctx.set_j(*dev)
        tuned = ctx.autotune(pgh.PGH_FAMILY_NEWTON_ALLPAIRS, dev[0], dev[1], dev[2], reps=2)
    timer = KernelTimer(torch)
    timing = {"on": False}

    def step():
        pgh.pgh_set_xmj(ctx.h, 0, n, *dev)
        pgh.pgh_set_n(ctx.h, n)
        if timing["on"]:
            with timer:
                pgh.pgh_calc_newton(ctx.h, n, dev[0], dev[1], dev[2], None, *out)
        else:
            pgh.pgh_calc_newton(ctx.h, n, dev[0], dev[1], dev[2], None, *out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    timing["on"] = True
    sec = time_steps(torch, step, args.steps, 0)
    kern_ms = timer.mean_ms()
    kern_all = timer.times_ms()
    variant = pgh.pgh_get_variant(ctx.h, pgh.PGH_FAMILY_NEWTON_ALLPAIRS)
    name = pgh.pgh_variant_name(pgh.PGH_FAMILY_NEWTON_ALLPAIRS, variant) if variant >= 0 else "default"
    refine = ctx.refine
    ctx.close()
    return {"n": n, "x": (x, y, z, m), "sec": sec, "kern_ms": kern_ms, "variant": variant,
            "variant_name": name, "autotuned": tuned is not None, "refine": refine,
            "kern_ms_median": float(np.median(kern_all)), "kern_ms_min": float(np.min(kern_all))}


REPLAYS = {"override": 0}


def graph_ms(torch, fn, reps, calls=1):
    """Captures `calls` consecutive calls of fn() in one graph (a hipGraph
    under ROCm) and returns the mean time per call in ms over `reps` replays,
    from events on the replay stream.  A replay of a one-call graph costs
    about 17 us of host time on this stack, so microsecond kernels are timed
    from graphs of several calls, where only the device's dispatch gaps remain
    between them."""
    reps = REPLAYS["override"] or reps
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
        fn()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(calls):
            fn()
    g.replay()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / (reps * calls)


CALLS_PER_GRAPH = 10


def call_times(torch, fn, reps):
    """Per-call ms from a graph of CALLS_PER_GRAPH calls (the rate the device
    sustains when the caller keeps it fed) and per replay of a one-call graph
    (which adds the host's replay cost)."""
    return {"ms_per_call": graph_ms(torch, fn, max(2, reps // CALLS_PER_GRAPH), CALLS_PER_GRAPH),
            "ms_per_replay_1call": graph_ms(torch, fn, reps)}


def newton_refined(torch, pgh, synth):
    """The headline workload (Plummer N = 262144, eps = 0.01) with one
    Newton-Raphson step after v_rsq_f32 (pgh_set_rsqrt_refine(1)), the
    literal form of the rsqrt refinement of Sec. 2: the variant the
    autotuner picks with the step on, kernel time from events on the launch
    stream (5 calls after 2)."""
    n = 262144
    x, y, z = synth.plummer(n, 102)
    m = synth.equal_masses(n)
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    out = [torch.empty(n, device="cuda") for _ in range(4)]
    ctx = pgh.Context(0)
    ctx.set_eps_to_all(0.01)
    ctx.set_rsqrt_refine(1)
    ctx.set_j(*dev)
    fam = pgh.PGH_FAMILY_NEWTON_ALLPAIRS
    v = ctx.autotune(fam, dev[0], dev[1], dev[2], reps=2)
    timer = KernelTimer(torch)
    for k in range(7):
        if k < 2:
            pgh.pgh_calc_newton(ctx.h, n, dev[0], dev[1], dev[2], None, *out)
            continue
        with timer:
            pgh.pgh_calc_newton(ctx.h, n, dev[0], dev[1], dev[2], None, *out)
    ms = timer.mean_ms()
    ctx.close()
    inter = float(n) * n
    return {"workload": "newton_allpairs_plummer_N262144_eps0.01_rsqrt_newton_step",
            "rsqrt_refine": 1, "kernel_variant": pgh.pgh_variant_name(fam, v), "kernel_ms": ms,
            "interactions_per_s": inter / (ms / 1e3),
            "frac_of_peak_38flop": NEWTON_FLOPS * inter / (ms / 1e3) / (PEAK_FP32_TFLOPS * 1e12)}


def newton_small(torch, pgh, synth):
    """Newton all-pairs at N = 1024 (Plummer, seed 101, eps = 1/64): a
    launch-bound size; the set_xmj + calc_newton pair, timed from graphs."""
    n = 1024
    x, y, z = synth.plummer(n, 101)
    m = synth.equal_masses(n)
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    ctx = pgh.Context(0)
    ctx.set_eps_to_all(1.0 / 64)
    out = [torch.empty(n, device="cuda") for _ in range(4)]

    def call():
        ctx.set_j(*dev)
        pgh.pgh_calc_newton(ctx.h, n, dev[0], dev[1], dev[2], None, *out)

    t = call_times(torch, call, 200)
    ctx.close()
    return {"workload": "newton_allpairs_plummer_N1024_eps1/64", **t,
            "interactions_per_s": n * n / (t["ms_per_call"] / 1e3)}


def grape5_host(torch, pgh, synth, n=262144):
    """The GRAPE-5-compatible host interface on the headline workload
    (Plummer N = 262144, eps = 0.01): g5_set_xmj + g5_calculate_force_on_x on
    host double arrays, wall-clock time per step including the conversions
    and PCIe transfers (the device-array entry points avoid those)."""
    x, y, z = synth.plummer(n, 102)
    xs = np.ascontiguousarray(np.stack([x, y, z], axis=1).astype(np.float64))
    m = synth.equal_masses(n).astype(np.float64)
    a = np.zeros((n, 3))
    p = np.zeros(n)
    pgh.g5_open()
    pgh.g5_set_eps_to_all(0.01)
    pgh.g5_set_n(n)

    def step():
        pgh.g5_set_xmj(0, n, xs, m)
        pgh.g5_calculate_force_on_x(xs, a, p, n)

    step()
    t0 = time.perf_counter()
    for _ in range(3):
        step()
    sec = (time.perf_counter() - t0) / 3
    pgh.g5_close()
    return {"workload": "grape5_host_arrays_plummer_N262144_eps0.01", "ms_per_step": sec * 1e3,
            "interactions_per_s_incl_pcie": float(n) * n / sec}


def ni_nj_sweep(torch, pgh, synth):
    """Throughput against group and list size (the small N_i / N_j regime of
    tree codes with individual time steps): lists of n_i i-particles (a
    Plummer sphere of 2^21, consecutive groups) against n_j j-particles
    (consecutive windows of the same sphere), eps = 1e-3, about 2^31
    interactions per launch (at most 131072 lists).  Each point runs the
    lists two ways: GRAPE-style, one pgh_set_xmj + pgh_calc_newton per list
    (ten lists captured in one graph, so the time per list is the device's,
    not Python's), and all lists in one persistent batched launch."""
    n = 1 << 21
    x, y, z = synth.plummer(n, 106)
    m = synth.equal_masses(n)
    d = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    ctx = pgh.Context(0)
    ctx.set_eps_to_all(1e-3)
    out = [torch.empty(n, device="cuda") for _ in range(4)]
    res = []
    for ni in (16, 64, 256, 1024):
        for nj in (64, 512, 4096):
            n_items = int(min(131072, n // ni, max(1, (1 << 31) // (ni * nj))))
            items = np.array([[k * ni, ni, (k * 7919) % (n - nj), nj] for k in range(n_items)],
                             np.int32)
            plan = ctx.plan(items, n, n)
            ms = graph_ms(torch, lambda: plan.newton(*d[:3], *d, out=out), 5)
            inter = float(plan.interactions)
            plan.free()
            # GRAPE-style calls: one list per call, j-memory = that list's window
            calls = [(int(items[k][0]), int(items[k][2])) for k in range(min(n_items, 10))]
            views = [([t[j0:j0 + nj] for t in d], [t[i0:i0 + ni] for t in d[:3]],
                      [t[i0:i0 + ni] for t in out]) for i0, j0 in calls]

            def grape_calls():
                for jv, iv, ov in views:
                    pgh.pgh_set_xmj(ctx.h, 0, nj, *jv)
                    pgh.pgh_set_n(ctx.h, nj)
                    pgh.pgh_calc_newton(ctx.h, ni, *iv, None, *ov)

            call_ms = graph_ms(torch, grape_calls, 20) / len(views)
            res.append({"n_i": ni, "n_j": nj, "lists": n_items,
                        "batched_interactions_per_s": inter / (ms / 1e3),
                        "per_call_interactions_per_s": ni * nj / (call_ms / 1e3),
                        "per_call_us": call_ms * 1e3})
    ctx.close()
    return res


def batched_newton(torch, pgh, synth):
    """Tree-style lists: 16384 (i-group, j-list) items over a Morton-sorted
    Plummer sphere of 2^22 particles, eps = 1e-3, i-groups uniform in
    [32, 256], j-lists log-normal (median 2000, clipped [200, 20000]),
    materialised; one persistent launch per step, replayed from a graph."""
    s = synth.tree_style_items(1 << 22, 16384, 104)
    di = [torch.from_numpy(a).cuda() for a in (s.xi, s.yi, s.zi)]
    dj = [torch.from_numpy(a).cuda() for a in (s.xj, s.yj, s.zj, s.mj)]
    ctx = pgh.Context(0)
    ctx.set_eps_to_all(1e-3)
    plan = ctx.plan(s.items, s.xi.size, s.xj.size)
    out = [torch.empty(s.xi.size, device="cuda") for _ in range(4)]
    fam = pgh.PGH_FAMILY_NEWTON_BATCH
    per = {}
    for v in range(pgh.pgh_variant_count(fam)):
        ctx.set_variant(fam, v)
        per[pgh.pgh_variant_name(fam, v)] = graph_ms(torch, lambda: plan.newton(*di, *dj, out=out), 10)
    inter = float(plan.interactions)
    plan.free()
    # the library's tuner: plans cut for 0.5, 1 and 2 times the resident
    # waves, plain and packed, every variant timed on each
    plan, tuned, scale = ctx.plan_tuned(s.items, s.xi.size, s.xj.size, fam, *di, *dj, reps=3)
    packed = plan.packed
    ms = graph_ms(torch, lambda: plan.newton(*di, *dj, out=out), 10)
    plan.free()
    ctx.close()
    rate = inter / (ms / 1e3)
    return {"workload": "newton_batched_tree_style_16384_lists_N4194304", "interactions": inter,
            "ms_per_launch": ms, "interactions_per_s": rate,
            "frac_of_peak_38flop": NEWTON_FLOPS * rate / (PEAK_FP32_TFLOPS * 1e12),
            "autotuned_variant": pgh.pgh_variant_name(fam, tuned),
            "autotuned_plan_waves_scale": scale, "autotuned_packing": packed,
            "ms_per_variant": per}


def useful_pairs(s, rcut):
    """Pairs of the lists closer than rcut (the ones with a non-zero force),
    counted on the host."""
    r2 = rcut * rcut
    count = 0
    for i0, ni, j0, nj in s.items:
        if ni == 0 or nj == 0:
            continue
        dx = s.xj[j0:j0 + nj][None, :] - s.xi[i0:i0 + ni][:, None]
        dy = s.yj[j0:j0 + nj][None, :] - s.yi[i0:i0 + ni][:, None]
        dz = s.zj[j0:j0 + nj][None, :] - s.zi[i0:i0 + ni][:, None]
        count += int(np.count_nonzero(dx * dx + dy * dy + dz * dz < r2))
    return count


def batched_table(torch, pgh, synth):
    """Cell-grid lists of a TreePM PP step: N = 262144 uniform in the unit
    periodic box, 64^3 cells, i-groups of 4^3 cells with their 6^3-cell halo
    (4096 lists; and 8^3-cell groups with a 10^3-cell halo, 512 lists),
    S2 PP shape rcut = 3/256, eps = 1/1280, E = 4, F = 6 (and F = 5).  Every
    tile shape of the batched kernel is timed on the default plan; the
    library's tuner (Context.plan_tuned: plan wave target x packing x tile shape)
    chooses, and its choice is reported with its per-call time from a graph
    of ten calls and per replay of a one-call graph; also the rate of useful
    pairs (closer than rcut)."""
    n = 262144
    rcut = 3.0 / 256
    x, y, z = synth.uniform_box(n, 103)
    m = synth.equal_masses(n)
    res = {}
    for block, F in ((4, 6), (8, 6), (4, 5)):
        s = synth.cell_grid_items(x, y, z, m, ncell=64, block=block)
        di = [torch.from_numpy(a).cuda() for a in (s.xi, s.yi, s.zi)]
        dj = [torch.from_numpy(a).cuda() for a in (s.xj, s.yj, s.zj, s.mj)]
        ctx = pgh.Context(0)
        ctx.build_table(4, F, rcut, eps=1.0 / 1280)
        plan = ctx.plan(s.items, n, s.xj.size)
        out = [torch.empty(n, device="cuda") for _ in range(3)]
        fam = pgh.PGH_FAMILY_TABLE_BATCH
        per = {}
        for v in range(pgh.pgh_variant_count(fam)):
            ctx.set_variant(fam, v)
            per[pgh.pgh_variant_name(fam, v)] = graph_ms(
                torch, lambda: plan.table(*di, *dj, out=out), 20, CALLS_PER_GRAPH)
        inter = float(plan.interactions)
        plan.free()
        # the library's tuner: plans cut for 0.5, 1 and 2 times the resident
        # waves, plain and packed, every variant timed on each
        plan, tuned, scale = ctx.plan_tuned(s.items, n, s.xj.size, fam, *di, *dj, reps=20)
        packed = plan.packed
        t = call_times(torch, lambda: plan.table(*di, *dj, out=out), 200)
        plan.free()
        ctx.close()
        ms = t["ms_per_call"]
        rate = inter / (ms / 1e3)
        useful = useful_pairs(s, rcut)
        res[f"block{block}" + ("" if F == 6 else f"_F{F}")] = {
            "workload": f"table_batched_cell_lists_N262144_E4F{F}_block{block}",
            "lists": int(len(s.items)), "interactions": inter, "useful_pairs": useful, **t,
            "interactions_per_s": rate, "useful_pairs_per_s": useful / (ms / 1e3),
            "frac_of_peak_20flop": TABLE_FLOPS * rate / (PEAK_FP32_TFLOPS * 1e12),
            "frac_of_peak_20flop_1call_replay":
                TABLE_FLOPS * inter / (t["ms_per_replay_1call"] / 1e3) / (PEAK_FP32_TFLOPS * 1e12),
            "autotuned_variant": pgh.pgh_variant_name(fam, tuned),
            "autotuned_plan_waves_scale": scale, "autotuned_packing": packed,
            "ms_per_call_per_variant": per}
    return res


def adjoint_newton(torch, pgh, synth):
    """Forward + backward of L = sum_i w_i . a_i over all pairs of a Plummer
    sphere of N = 65536 (seed 105), eps = 0.01, w ~ N(0, 1)^3: kernel-only
    times of pgh_calc_newton and pgh_newton_allpairs_bwd, and the time of the
    same through torch.autograd."""
    n = 65536
    x, y, z = synth.plummer(n, 105)
    m = synth.equal_masses(n)
    w = [torch.from_numpy(a).cuda() for a in synth.weights(n, 205)]
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    ctx = pgh.Context(0)
    ctx.set_eps_to_all(0.01)
    ctx.set_j(*dev)
    out = [torch.empty(n, device="cuda") for _ in range(4)]
    grads = [torch.empty(n, device="cuda") for _ in range(4)]
    eps2 = float(np.float32(0.01) ** 2)
    tf, tb = KernelTimer(torch), KernelTimer(torch)
    for it in range(8):
        with tf:
            pgh.pgh_calc_newton(ctx.h, n, dev[0], dev[1], dev[2], None, *out)
        with tb:
            pgh.pgh_newton_allpairs_bwd(ctx.h, n, *dev, eps2, *w, *grads)
    fwd, bwd = tf.mean_ms(), tb.mean_ms()
    # through torch.autograd (includes packing and allocation)
    req = [t.clone().requires_grad_(True) for t in dev]

    def fwd_only():
        with torch.no_grad():
            pgh.newton_allpairs(*req, 0.01, ctx)

    def fwd_bwd():
        ax, ay, az, _ = pgh.newton_allpairs(*req, 0.01, ctx)
        (ax * w[0] + ay * w[1] + az * w[2]).sum().backward()

    # host-timed: the fastest of three runs of five steps each, so that a
    # host stall in one run does not decide the ratio
    t_f = min(time_steps(torch, fwd_only, 5, 2) for _ in range(3))
    t_fb = min(time_steps(torch, fwd_bwd, 5, 2) for _ in range(3))
    ctx.close()
    inter = float(n) * n
    return {"workload": "newton_allpairs_adjoint_plummer_N65536_eps0.01",
            "fwd_kernel_ms": fwd, "bwd_kernel_ms": bwd,
            "fwd_plus_bwd_over_fwd_kernel": (fwd + bwd) / fwd,
            "fwd_plus_bwd_over_fwd_autograd": t_fb / t_f,
            "bwd_interactions_per_s": inter / (bwd / 1e3)}


def adjoint_table(torch, pgh, synth):
    """Table-force forward and adjoint on cell lists: N = 65536 uniform in the
    unit periodic box, 64^3 cells, 8^3-cell groups, S2 PP shape (rcut = 3/256,
    eps = 1/1280, E = 4, F = 6); the adjoint with respect to the table entries
    and masses, and also with the i- and j-position gradients (two passes over
    the pairs, or one with the moments kept by the forward); per call from
    graphs of ten calls."""
    n = 65536
    x, y, z = synth.uniform_box(n, 105)
    m = synth.equal_masses(n)
    s = synth.cell_grid_items(x, y, z, m, ncell=64, block=8)
    di = [torch.from_numpy(a).cuda() for a in (s.xi, s.yi, s.zi)]
    dj = [torch.from_numpy(a).cuda() for a in (s.xj, s.yj, s.zj, s.mj)]
    w = [torch.from_numpy(a).cuda() for a in synth.weights(n, 305)]
    ctx = pgh.Context(0)
    table = ctx.build_table(4, 6, 3.0 / 256, eps=1.0 / 1280)
    plan = ctx.plan(s.items, n, s.xj.size)
    out = [torch.empty(n, device="cuda") for _ in range(3)]
    gt = torch.empty(table.size, device="cuda")
    gm = torch.empty(s.xj.size, device="cuda")
    f_ms = graph_ms(torch, lambda: plan.table(*di, *dj, out=out), 10, CALLS_PER_GRAPH)
    b_ms = graph_ms(torch, lambda: pgh.pgh_batch_table_bwd(ctx.h, plan.h, *di, *dj, *w, gt, gm), 10,
                    CALLS_PER_GRAPH)
    gi = [torch.empty(n, device="cuda") for _ in range(3)]
    gj = [torch.empty(s.xj.size, device="cuda") for _ in range(3)]
    bx_ms = graph_ms(torch, lambda: pgh.pgh_batch_table_bwd(ctx.h, plan.h, *di, *dj, *w, gt, gm,
                                                            *gi, *gj), 10, CALLS_PER_GRAPH)
    # the training path for position gradients: a forward that keeps the
    # i-side moments, a backward that forms the i-side gradient from them
    mom = torch.empty(7 * n, device="cuda")
    fm_ms = graph_ms(torch, lambda: pgh.pgh_batch_table_moments(ctx.h, plan.h, *di, *dj, *out, mom),
                     10, CALLS_PER_GRAPH)
    bm_ms = graph_ms(torch, lambda: pgh.pgh_batch_table_bwd_moments(
        ctx.h, plan.h, *di, *dj, *w, mom, gt, gm, *gi, *gj), 10, CALLS_PER_GRAPH)
    inter = float(plan.interactions)
    plan.free()
    ctx.close()
    return {"workload": "table_adjoint_cell_lists_N65536_8cube_groups_E4F6",
            "interactions": inter, "fwd_ms": f_ms, "bwd_ms": b_ms,
            "fwd_plus_bwd_over_fwd": (f_ms + b_ms) / f_ms,
            "bwd_with_positions_ms": bx_ms,
            "fwd_plus_bwd_with_positions_over_fwd": (f_ms + bx_ms) / f_ms,
            "fwd_with_moments_ms": fm_ms, "bwd_with_positions_from_moments_ms": bm_ms,
            # (forward keeping the moments + backward with every gradient) over the plain forward
            "fwd_moments_plus_bwd_with_positions_over_fwd": (fm_ms + bm_ms) / f_ms}


def table_allpairs(torch, pgh, synth):
    """Secondary: the table force on the same kind of call, N = 65536 uniform
    particles in a box of side 0.25 with the S2 PP shape (rcut = 3/256,
    eps = 1/1280, E = 4, F = 6), all pairs evaluated (most beyond rcut)."""
    n = 65536
    x, y, z = synth.uniform_box(n, 103, box=0.25)
    m = synth.equal_masses(n)
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    ctx = pgh.Context(0)
    ctx.build_table(4, 6, 3.0 / 256, eps=1.0 / 1280)
    ctx.set_j(*dev)
    out = [torch.empty(n, device="cuda") for _ in range(3)]
    fam = pgh.PGH_FAMILY_TABLE_ALLPAIRS
    per = {}
    # ten untimed calls first: after the idle table upload the first
    # launches run up to a quarter slower
    for _ in range(10):
        pgh.pgh_calc_table(ctx.h, n, dev[0], dev[1], dev[2], *out, None)
    for v in range(pgh.pgh_variant_count(fam)):
        ctx.set_variant(fam, v)
        pgh.pgh_calc_table(ctx.h, n, dev[0], dev[1], dev[2], *out, None)  # untimed
        t = KernelTimer(torch)
        for _ in range(4):
            with t:
                pgh.pgh_calc_table(ctx.h, n, dev[0], dev[1], dev[2], *out, None)
        per[pgh.pgh_variant_name(fam, v)] = t.mean_ms()
    # with the potential from a second table (the same shape's potential is
    # not needed for timing: any table on the same bins costs the same)
    ctx.build_pot_table(lambda r: -1.0 / (r + 1.0 / 1280) + 1.0 / (3.0 / 256 + 1.0 / 1280))
    phi = torch.empty(n, device="cuda")
    pgh.pgh_calc_table(ctx.h, n, dev[0], dev[1], dev[2], *out, phi)  # untimed
    tp = KernelTimer(torch)
    for _ in range(4):
        with tp:
            pgh.pgh_calc_table(ctx.h, n, dev[0], dev[1], dev[2], *out, phi)
    ctx.set_variant(fam, -1)  # the built-in default (the paper's table form)
    timer = KernelTimer(torch)

    def step():
        with timer:
            pgh.pgh_calc_table(ctx.h, n, dev[0], dev[1], dev[2], *out, None)

    sec = time_steps(torch, step, 10, 2)
    ms = timer.mean_ms()
    # the largest tables (wider workgroups: the table fills most of a CU's
    # LDS), the (H, G1) form: 2^14 nodes, and 2^13 with the potential
    names = [pgh.pgh_variant_name(fam, v) for v in range(pgh.pgh_variant_count(fam))]
    ctx.set_variant(fam, names.index("ki=1 jt=256 u=4 htab"))
    large = {}
    for F, with_phi in ((10, False), (9, True)):
        ctx.build_table(4, F, 3.0 / 256, eps=1.0 / 1280)
        if with_phi:
            ctx.build_pot_table(lambda r: -1.0 / (r + 1.0 / 1280) + 1.0 / (3.0 / 256 + 1.0 / 1280))
        for _ in range(3):  # untimed
            pgh.pgh_calc_table(ctx.h, n, dev[0], dev[1], dev[2], *out, phi if with_phi else None)
        tl = KernelTimer(torch)
        for _ in range(4):
            with tl:
                pgh.pgh_calc_table(ctx.h, n, dev[0], dev[1], dev[2], *out, phi if with_phi else None)
        large[f"E4F{F}" + ("_with_potential" if with_phi else "")] = tl.mean_ms()
    ctx.close()
    inter = float(n) * n
    return {"workload": "table_allpairs_uniform_N65536_E4F6", "interactions_per_s": inter / (ms / 1e3),
            "kernel_ms": ms, "step_ms": sec * 1e3,
            "frac_of_peak_20flop": TABLE_FLOPS * inter / (ms / 1e3) / (PEAK_FP32_TFLOPS * 1e12),
            "ms_per_variant": per, "kernel_ms_with_potential_last_variant": tp.mean_ms(),
            "kernel_ms_large_tables_htab": large}


def tree_code(torch, pgh, synth, sizes=(1 << 20, 1 << 22), n_crit=64,
              models=("plummer", "king9")):
    """The tree code of Sec. 5 (Fig. 10): forces and potentials of every
    particle of a Plummer sphere (scale radius 1) and of a King model with
    W0 = 9 (King radius 1) with the device Barnes-Hut tree, theta = 0.75,
    leaves of at most 8 particles, i-groups of at most n_crit, eps = 1/512,
    monopole and quadrupole pseudo-particles.  Wall-clock per phase, each
    call synchronous except the force (timed with events, then waited for):
    build (keys, sort, octree, moments, groups), walk (both passes and the
    batched plan of the lists), force (batched Newton, results written in
    the input order).  Median of 3 after one warm-up."""
    res = {}
    ctx = pgh.Context(0)
    ctx.set_eps_to_all(1.0 / 512)
    cases = [(model, n) for model in models for n in sizes]
    for model, n in cases:
        x, y, z = synth.plummer(n, 330) if model == "plummer" else synth.king(n, 331, 9.0)
        m = synth.equal_masses(n)
        d = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
        t = ctx.tree()
        per_n = {}
        for quad in (False, True):
            t.build(*d, n_leaf=8, n_crit=n_crit, quad=quad)
            t.walk(0.75)
            out = t.newton()
            torch.cuda.synchronize()
            tb, tw, tt = [], [], []
            timer = KernelTimer(torch)
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                t.build(*d, n_leaf=8, n_crit=n_crit, quad=quad)
                t1 = time.perf_counter()
                t.walk(0.75)
                t2 = time.perf_counter()
                with timer:
                    t.newton(out=out)
                torch.cuda.synchronize()
                t3 = time.perf_counter()
                tb.append(t1 - t0)
                tw.append(t2 - t1)
                tt.append(t3 - t0)
            tf = timer.times_ms()
            st = t.stats()
            inter = float(st["interactions"])
            f_ms = float(np.median(tf))
            rate = inter / (f_ms / 1e3)
            per_n["quadrupole" if quad else "monopole"] = {
                "build_ms": 1e3 * float(np.median(tb)), "walk_and_plan_ms": 1e3 * float(np.median(tw)),
                "force_ms": f_ms, "total_ms": 1e3 * float(np.median(tt)),
                "n_nodes": st["n_nodes"], "n_groups": st["n_groups"], "depth": st["depth"],
                "max_frontier": st["max_frontier"],
                "list_entries": st["n_entries"], "mean_list_length": st["n_entries"] / max(1, st["n_groups"]),
                "interactions": inter, "force_interactions_per_s": rate,
                "force_frac_of_peak_38flop": NEWTON_FLOPS * rate / (PEAK_FP32_TFLOPS * 1e12)}
        t.free()
        res[f"{model}_N{n}"] = per_n
        del d
    ctx.close()
    return {"workload": f"tree_code_theta0.75_nleaf8_ncrit{n_crit}_eps1/512", **res}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1).", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1203_4037_amd as pgh
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    REPLAYS["override"] = args.replays
    if args.only_extra:
        extras = {"newton_small": newton_small, "newton_refined": newton_refined,
                  "table_allpairs": table_allpairs,
                  "newton_batched": batched_newton, "table_batched": batched_table,
                  "adjoint_newton": adjoint_newton, "adjoint_table": adjoint_table,
                  "ni_nj_sweep": ni_nj_sweep, "grape5_host": grape5_host,
                  "tree_code": lambda t, p, s: tree_code(t, p, s, n_crit=1024)}
        if args.only_extra not in extras:
            print(f"unknown workload {args.only_extra}; one of {sorted(extras)}", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({args.only_extra: extras[args.only_extra](torch, pgh, synth)}))
        return
    r = newton_allpairs(torch, pgh, synth, args)
    if args.copy_calibration > 0:
        src = torch.empty(args.copy_calibration << 18, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = r["n"]
    inter = float(n) * n
    value = inter / r["sec"]
    achieved = NEWTON_FLOPS * inter / (r["kern_ms"] / 1e3) / 1e12
    cnt = counters_for(r["variant_name"], r["refine"])
    hw_flops = cnt["valu_flops_per_interaction"] if cnt else None
    hw_tflops = hw_flops * inter / (r["kern_ms"] / 1e3) / 1e12 if hw_flops else None
    line = {
        "metric": "interactions/sec on 1 MI355X (Newton, LUT) + % FP32 VALU peak; batched vs all-pairs; fwd+bwd/fwd",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"newton_allpairs_plummer_N{n}_eps0.01", "n_i": n, "n_j": n,
                   "eps": 0.01, "seed": 102, "interactions_per_step": inter,
                   "parallelism": "single_gpu", "kernel_variant": r["variant_name"],
                   "autotuned": r["autotuned"], "rsqrt_refine": r["refine"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(r["variant_name"], r["refine"]),
                     "traffic_unit": "bytes/launch",
                     "kernel": "k_newton_allpairs",
                     # HIP events around pgh_calc_newton on its stream: the kernel and,
                     # when the j-range is split, k_combine_split (a few microseconds)
                     "kernel_ms": r["kern_ms"],
                     "kernel_ms_median": r["kern_ms_median"], "kernel_ms_min": r["kern_ms_min"],
                     "flops_per_interaction": NEWTON_FLOPS,
                     # the FP32 flops the VALU counters count for this kernel (FMA = 2;
                     # 21 per interaction, not the paper's 38) against the same peak;
                     # null when the counters were taken on other sources
                     "valu_flops_per_interaction": hw_flops,
                     "valu_tflops": hw_tflops,
                     "valu_frac_of_peak": (hw_tflops / PEAK_FP32_TFLOPS if hw_tflops else None)},
    }
    if not args.no_extras:
        ex = {"newton_refined": newton_refined(torch, pgh, synth),
              "newton_small": newton_small(torch, pgh, synth),
              "table_allpairs": table_allpairs(torch, pgh, synth),
              "newton_batched": batched_newton(torch, pgh, synth),
              "table_batched": batched_table(torch, pgh, synth),
              "adjoint_newton": adjoint_newton(torch, pgh, synth),
              "adjoint_table": adjoint_table(torch, pgh, synth),
              "ni_nj_sweep": ni_nj_sweep(torch, pgh, synth),
              "grape5_host": grape5_host(torch, pgh, synth),
              "tree_code": tree_code(torch, pgh, synth, n_crit=1024)}
        ex["batched_over_allpairs"] = ex["newton_batched"]["interactions_per_s"] / value
        line["extras"] = ex
    if not args.no_cpu:
        x, y, z, m = r["x"]
        line["cpu_baseline"] = cpu_baseline(x, y, z, m, 0.01, args.cpu_seconds, synth)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
