"""Throughput of the fused FP32 hybrid-LBM step on one MI355X.

Workload: decaying compressible turbulence on an 8192 x 8192 periodic grid
(seeded random-phase solenoidal velocity, E(k) ~ k^4 exp(-2 (k/8)^2),
turbulent Mach 0.5, rho = 1, theta = 240/1183), nu = 1e-3, sigma = 0, FP32
storage.  A step is the whole fused update of every node (collision,
correction term, streaming and entropy update); on this periodic grid the
library advances two steps per kernel launch (the two-step sweep reads the
state once and writes it once per two steps).

Prints ONE JSON line: MLUPS (million lattice updates per second), the HBM
roofline of the step kernel, the FP64 CPU oracle timed on a bounded sample of
the same workload on the host cores, and (second part of the metric) the
learned closure: a coarse 256^2 HLBM corrected by the BF16-MFMA network,
trained on the GPU on 4x-restricted 1024^2 runs, against the plain ladder
256^2 .. 1024^2 -- wall time of the plain run that reaches the learned run's
density error, divided by the learned run's wall time.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("HLBM MLUPS & % HBM roofline @8192² FP32; learned-vs-plain time at equal L2 "
          "error")
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s
BYTES_PER_NODE = 80            # per lattice update: read 9 populations + s, write 9 + s, FP32
# sources that decide the step kernels and their launch shapes (tile defaults)
KERNEL_SRCS = [os.path.join(ROOT, "paper_2002_03644_amd", "csrc", f)
               for f in ("hlbm_device.hpp", "hlbm_step2.hpp", "hlbm_launch.hpp")]
# HBM counter summaries of the dominant kernel, per steps per launch
TRAFFIC_FILES = {1: os.path.join(ROOT, "profiles", "k_step_f32_turbulence8192_traffic.txt"),
                 2: os.path.join(ROOT, "profiles", "k_step2_f32_turbulence8192_traffic.txt")}
KERNEL_NAMES = {1: "hlbm::f32::k_step<{w}>", 2: "hlbm::f32::k_step2<{w}>"}


def code_text(src: str) -> str:
    """C++ source without comments, string-free by construction here, with
    runs of whitespace collapsed: the part of a file that the compiler sees
    as code, so that editing a comment leaves the hash alone."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_hash() -> str:
    """First 16 hex digits of the SHA-256 of the step kernels' code (see
    code_text), the key the committed counter summaries are checked by."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(nodes: int, spl: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    the kernel that does `spl` steps per launch (lines `key: value`), if it
    was taken on the current kernel source at this grid size; else None."""
    try:
        with open(TRAFFIC_FILES[spl]) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_source_sha256_16") != kernel_hash() or kv.get("nodes") != str(nodes):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def f64_same_config(n, fields, tile_w, tile_h, steps=100, keep=None):
    """The same workload in FP64 (160 algorithmic bytes per node), timed over
    `steps` steps after 5 warm-up steps, for context beside the FP32 line.
    With `keep` (a list) the solver is appended to it instead of freed."""
    import torch

    from paper_2002_03644_amd import Params, Solver, launch_shape
    r, u, v, t = fields
    S = Solver(Params(n, n, dtype="f64", mu=1e-3, sigma=0.0, tile_w=tile_w, tile_h=tile_h),
               r, u, v, theta=t)
    S.step(5)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    S.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    code, _ = S.status()
    if keep is not None:
        keep.append(S)
    del S
    if keep is None:
        torch.cuda.empty_cache()
    gbs = 2 * BYTES_PER_NODE * n * n / (ms / 1e3) / 1e9
    tw, th = launch_shape(Params(n, n, dtype="f64", tile_w=tile_w, tile_h=tile_h))
    return {"mlups": round(n * n / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "achieved": round(gbs, 1), "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "steps": steps, "status_after": int(code), "tile_w": tw, "tile_h": th}


def gpu_same_window(oracle_mlups, n=1024, steps=150):
    """The GPU library on the oracle's sample (the same 1024^2 window of the
    turbulence recipe, 150 steps), FP32 and FP64, for a side-by-side ratio."""
    import torch

    import hlbm_inputs as hi
    from paper_2002_03644_amd import Params, Solver
    r, u, v, t = hi.turbulence(n, 0.5, hi.THETA_PAPER, seed=0)
    out = {}
    for dt in ("f32", "f64"):
        S = Solver(Params(n, n, dtype=dt, mu=1e-3, sigma=0.0), r, u, v, theta=t)
        S.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.step(steps)
        torch.cuda.synchronize()
        out[f"{dt}_mlups"] = round(n * n * steps / (time.perf_counter() - t0) / 1e6, 1)
        del S
    out["f64_over_oracle"] = round(out["f64_mlups"] / oracle_mlups, 1)
    out["f32_over_oracle"] = round(out["f32_mlups"] / oracle_mlups, 1)
    out["sample"] = f"{n}x{n} window, {steps} steps, default tiles"
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    """Host CPU model name (Linux), or 'unknown'."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_sample=1024, steps=150):
    """The FP64 oracle on an n_sample^2 periodic window of the same
    turbulence recipe, timed on the host cores (steady-state steps only)."""
    import numpy as np

    import hlbm_inputs as hi
    import oracle
    r, u, v, t = hi.turbulence(n_sample, 0.5, hi.THETA_PAPER, seed=0)
    S = oracle.OracleSolver(oracle.OracleParams(n_sample, n_sample, mu=1e-3, sigma=0.0),
                            r, u, v, theta=t)
    S.step(1)
    cores = oracle.threads()
    t0 = time.perf_counter()
    S.step(steps)
    dt = time.perf_counter() - t0
    del S
    # one thread, on a 256^2 window of the same recipe
    n1, steps1 = 256, 30
    r, u, v, t = hi.turbulence(n1, 0.5, hi.THETA_PAPER, seed=0)
    S1 = oracle.OracleSolver(oracle.OracleParams(n1, n1, mu=1e-3, sigma=0.0), r, u, v, theta=t)
    oracle.threads(1)
    S1.step(1)
    t1 = time.perf_counter()
    S1.step(steps1)
    dt1 = time.perf_counter() - t1
    oracle.threads(cores)
    return {"value": round(n_sample * n_sample * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{n_sample}x{n_sample} periodic window of the same turbulence recipe, "
                      f"{steps} steps after 1 warm-up step, FP64, {dt:.1f} s",
            "single_thread": {"value": round(n1 * n1 * steps1 / dt1 / 1e6, 3), "unit": "MLUPS",
                              "sample": f"{n1}x{n1} window, {steps1} steps, {dt1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--tile-w", type=int, default=0)
    ap.add_argument("--tile-h", type=int, default=0)
    ap.add_argument("--every", type=int, default=1,
                    help="closure workload: plain steps per correction")
    ap.add_argument("--batch-kernel", default="strips", choices=["strips", "tiles"],
                    help="batch and closure workloads with --tile-w/--tile-h: the kernel "
                         "those name")
    ap.add_argument("--steps-per-launch", type=int, default=0, choices=[0, 1, 2],
                    help="0: the library's plan (two steps per launch here), 1 or 2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true",
                    help="skip the FP64 run of the same workload (100 steps)")
    ap.add_argument("--map-dtype", default="f64", choices=["f32", "f64"],
                    help="precision of the vortex-map workload")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-closure part (training + evaluation, about a minute)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 2 GiB device copy (counter calibration)")
    ap.add_argument("--workload", default="turbulence8192",
                    choices=["turbulence8192", "batch256", "closure", "vortex-map", "couette"],
                    help="batch256: the 256-domain batch (one persistent launch per step, "
                         "graph-replayed), reported as aggregate MLUPS of the domains still "
                         "active at the end; closure: the corrected coarse step of the "
                         "learned closure (8 x 256^2) and the network's training step; "
                         "vortex-map: the sigma x Mach isentropic-vortex study of Sec. 4.2 "
                         "(200^2, 50 convective times, 11 x 11 runs plus the original model); "
                         "couette: the thermal Couette flow of Sec. 4.4 on the 2 x 100 "
                         "channel to steady state, and the cost of walls on an 8192^2 channel")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is described in the design notes but not implemented", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch256":
        return bench_batch(args)
    if args.workload == "closure":
        return bench_closure(args)
    if args.workload == "vortex-map":
        return bench_vortex_map(args)
    if args.workload == "couette":
        return bench_couette(args)

    import numpy as np
    import torch

    import hlbm_inputs as hi
    from paper_2002_03644_amd import Params, Solver, launch_plan

    n = args.n
    print(f"[bench] generating {n}x{n} turbulence", file=sys.stderr, flush=True)
    r, u, v, t = hi.turbulence(n, 0.5, hi.THETA_PAPER, seed=0)
    params = Params(n, n, dtype="f32", mu=1e-3, sigma=0.0, tile_w=args.tile_w,
                    tile_h=args.tile_h, steps_per_launch=args.steps_per_launch)
    spl, tile_w, tile_h = launch_plan(params)
    dev = torch.device("cuda:0")
    fields = [torch.from_numpy(a.astype(np.float32)).to(dev) for a in (r, u, v, t)]
    S = Solver(params, *fields[:3], theta=fields[3], device=dev)
    del fields
    torch.cuda.synchronize()
    # The library copy of the step's bytes and the FP64 run of the same
    # workload (both reported below) run before the FP32 window, the FP64
    # steps last and with their solver kept until after the window (no
    # allocation or free in between): after host-side set-up, idle time or
    # the memory-bound copy, the first step launches run up to 30 % slower for
    # about 20 ms while the clocks settle under the compute-heavy load, which
    # a short timed window would otherwise measure instead of the kernel.
    stream_ref = copy_reference(n, dev)
    held = []
    f64 = None if args.no_f64 else f64_same_config(n, (r, u, v, t), 0, 0, keep=held)
    print("[bench] warmup", file=sys.stderr, flush=True)
    S.step(args.warmup)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    S.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps
    nodes = n * n
    mlups = nodes * args.steps / (ms_total / 1e3) / 1e6
    code, max_cfl = S.status()
    print(f"[bench] {ms_per_step:.4f} ms/step, {mlups:.0f} MLUPS, wall {wall:.2f} s, "
          f"status {code}, max CFL {max_cfl:.3f}", file=sys.stderr, flush=True)

    # the dominant kernel does `spl` lattice updates of every node per
    # launch; its algorithmic bytes per launch are 80 B x nodes x spl, and
    # its average launch duration is the timed region over its launches
    launches = args.steps // spl
    bytes_per_launch = BYTES_PER_NODE * nodes * spl
    ms_per_launch = ms_per_step * spl
    achieved = bytes_per_launch / (ms_per_launch / 1e3) / 1e9
    traffic = measured_traffic(nodes, spl) if args.steps % spl == 0 else None
    roofline = {"bound": "hbm", "kernel": KERNEL_NAMES[spl].format(w=tile_w),
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "steps_per_launch": spl, "launches": launches,
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "ms_per_launch": round(ms_per_launch, 5)}

    if args.copy_calibration:
        # a plain elementwise copy kernel moving 2 GiB in and 2 GiB out, whose
        # counter readings calibrate FETCH_SIZE / WRITE_SIZE
        a = torch.zeros(2 ** 29, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    del S, held
    torch.cuda.empty_cache()
    stream_ref["step_frac_of_copy"] = round(achieved / stream_ref["achieved"], 4)
    del r, u, v, t
    learned = None if args.no_learned else learned_closure()
    torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
        cpu["gpu_same_window"] = gpu_same_window(cpu["value"])

    out = {"metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"decaying compressible turbulence {n}x{n} periodic, "
                                  "Ma_t 0.5, nu 1e-3, sigma 0, FP32 storage",
                      "nx": n, "ny": n, "global_batch": 1, "parallelism": "none",
                      "steps_per_launch": spl, "tile_w": tile_w, "tile_h": tile_h,
                      "tiles_given": bool(params.tile_w and params.tile_h),
                      "status_after": int(code)},
           "roofline": roofline, "cpu_baseline": cpu, "stream_reference": stream_ref,
           "f64": f64, "device": torch.cuda.get_device_name(0),
           "learned_closure": learned}
    print(json.dumps(out), flush=True)


def copy_reference(n, dev):
    """A library elementwise copy moving the step kernel's algorithmic bytes
    (ten FP32 planes of n^2 read, ten written), as a practical-bandwidth
    reference for the roofline fraction."""
    import torch
    a = torch.zeros(10, n * n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        torch.mul(a, 1.0001, out=b)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    reps = 10
    for _ in range(reps):
        torch.mul(a, 1.0001, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    gbs = 80.0 * n * n / (ms / 1e3) / 1e9
    return {"kernel": "torch.mul elementwise copy, 10 planes in / 10 out", "ms": round(ms, 4),
            "achieved": round(gbs, 1), "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


def learned_closure():
    """Train the closure on 64 seeds, evaluate on 8 held-out seeds (all on the
    GPU); report the time at equal density error and the two targets."""
    import torch

    from paper_2002_03644_amd import learned as L
    setup = L.ClosureSetup()
    say = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    net, rec = L.fit(setup, steps=20000, batch=32, lr=2e-3, clip=4.0, log=say)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    ev = L.evaluate(net, setup)
    nc, nf = setup.coarse_n, setup.fine_n
    ratio = ev.time_at_equal_error()
    say(f"[bench] learned closure: e {ev.e_learned:.4f} vs plain {ev.e_plain}, "
        f"t {ev.t_learned * 1e3:.1f} ms vs {ev.t_plain}")
    return {"metric": "learned-vs-plain time at equal density L2 error",
            "value": None if ratio is None else round(ratio, 3), "unit": "x",
            "higher_is_better": True,
            "n_equal_error": None if ev.n_equal_error() is None else round(ev.n_equal_error(), 1),
            "e_learned": round(ev.e_learned, 5),
            "e_plain": {str(k): round(v, 5) for k, v in sorted(ev.e_plain.items())},
            "t_learned_ms": round(ev.t_learned * 1e3, 3),
            "t_plain_ms": {str(k): round(v * 1e3, 3) for k, v in sorted(ev.t_plain.items())},
            "speedup_vs_fine": round(ev.t_plain[nf] / ev.t_learned, 3),
            "target_error_within_2x_plain512": bool(ev.e_learned <= 2 * ev.e_plain[512]),
            "target_10x_faster_than_fine": bool(ev.t_learned <= ev.t_plain[nf] / 10),
            "diverged": {str(k): v for k, v in ev.diverged.items()},
            "train": {"pairs": rec["pairs"], "adam_steps": 20000, "batch": 32, "lr": 2e-3,
                      "final_loss": round(rec["loss"][-1][1], 5), "fit_s": round(fit_s, 1),
                      "correction_every": setup.every},
            "workload": f"decaying turbulence, Ma_t {setup.mach_range[0]}-{setup.mach_range[1]}, "
                        f"fine {nf}^2 (mu {setup.mu_fine}) restricted {setup.factor}x to {nc}^2; "
                        f"train seeds {len(setup.train_seeds)}, eval seeds "
                        f"{len(setup.eval_seeds)} batched, {setup.coarse_steps} coarse steps, "
                        "error = ||rho - rho_fine|| / ||rho_fine - mean|| over checkpoints "
                        f"{list(setup.checkpoints)}, times hipGraph-replayed"}


def bench_closure(args):
    """Corrected coarse steps of 8 periodic 256^2 domains (one HLBM step, the
    moments, the fused network and the correction per step, graph-replayed)
    and training steps of the network on batches of 16 fields; untrained
    network (the timing does not depend on the weights)."""
    import numpy as np
    import torch

    from paper_2002_03644_amd import CNN, BatchSolver
    from paper_2002_03644_amd import learned as L
    setup = L.ClosureSetup()
    nc = setup.coarse_n
    seeds = list(setup.eval_seeds)
    fields, params = [], []
    for s_ in seeds:
        r, u, v, t = L.fine_initial(s_, setup)
        f = setup.factor
        fields.append(tuple(np.ascontiguousarray(a[::f, ::f]) for a in (r, u, v, t)))
        params.append(L._params(nc, setup.mu_coarse, float(t[0, 0]), setup))
    B = BatchSolver(params, fields)
    if args.tile_w and args.tile_h:  # a given shape (profiling runs), else the autotuner's
        B.set_tile(args.tile_w, args.tile_h, kernel=args.batch_kernel)
        bk, tw, th = args.batch_kernel, args.tile_w, args.tile_h
    else:
        bk, tw, th = B.autotune(steps=10)
    net = CNN(len(seeds), nc, nc, L.initial_params(0))
    net.set_norm(np.array([1, 0, 0, 0.2], np.float32), np.array([0.1, 0.1, 0.1, 0.01], np.float32),
                 np.zeros(4, np.float32), np.array([1e-3, 1e-3, 1e-3, 1e-4], np.float32))
    net.set_output_clip(4.0)

    def timed(fn, stream):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    k = args.every
    cycles = max(1, args.steps // k)
    B.closure_step(net, max(2, args.warmup), every=k, graph=True)
    ms_c = timed(lambda: B.closure_step(net, cycles, every=k, graph=True), B.stream) / (cycles * k)
    B.step(max(2, args.warmup), graph=True)
    ms_p = timed(lambda: B.step(args.steps, graph=True), B.stream)
    Y = torch.randn(64, 4, nc, nc, device="cuda")
    D = torch.randn(64, 4, nc, nc, device="cuda")
    trn = CNN(16, nc, nc, L.initial_params(0))
    idx = torch.arange(16, dtype=torch.int32, device="cuda")
    nt = max(10, args.steps // 10)
    trn.train_step(Y, D, 1e-3, idx=idx)
    ms_t = timed(lambda: [trn.train_step(Y, D, 1e-3, idx=idx) for _ in range(nt)],
                 torch.cuda.current_stream())
    fwd_flop = 2.0 * nc * nc * 9 * (4 * 32 + 32 * 32 + 32 * 4)
    # the fused inference kernel alone: one launch per forward call
    x = torch.randn(len(seeds), 4, nc, nc, device="cuda") * 0.01
    y = torch.empty_like(x)
    nf = max(20, args.steps)
    net.forward(x, out=y)
    ms_f = timed(lambda: [net.forward(x, out=y) for _ in range(nf)], torch.cuda.current_stream())
    tflops = fwd_flop * len(seeds) / (ms_f / nf / 1e3) / 1e12
    out = {"metric": "corrected coarse step time (8 x 256^2)"
                     + ("" if k == 1 else f", one correction per {k} steps"),
           "value": round(ms_c * 1e3, 2), "unit": "us/step", "n_gpus": 1,
           "steps": cycles * k, "warmup": args.warmup,
           "ms_per_step": round(ms_c, 5), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "8 periodic 256^2 turbulence domains, learned closure",
                      "correction_every": k, "batch_kernel": bk, "tile_w": tw, "tile_h": th},
           "plain_step_us": round(ms_p / args.steps * 1e3, 2),
           "train_step_us_batch16": round(ms_t / nt * 1e3, 1),
           "network_flop_per_field": fwd_flop,
           "cnn_forward_us": round(ms_f / nf * 1e3, 2),
           "roofline": {"bound": "mfma", "kernel": "k_cnn_fused", "achieved": round(tflops, 1),
                        "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tflops / 2500.0, 4),
                        "traffic": None},
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_vortex_map(args):
    """The sigma x Mach map of the convected isentropic vortex (FP64 by
    default), one batch (11 sigma values + the original model) per Mach
    number."""
    from paper_2002_03644_amd import studies
    say = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    res = studies.sigma_mach_map(log=say, dtype=args.map_dtype)
    summ = studies.map_summary(res)
    out = {"metric": "sigma x Mach vortex map: aggregate lattice updates per second",
           "value": round(res.node_updates / res.seconds / 1e6, 1), "unit": "MLUPS",
           "n_gpus": 1, "steps": int(sum(res.steps.values())), "warmup": 0,
           "ms_per_step": round(res.seconds * 1e3 / sum(res.steps.values()), 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.map_dtype, "data": "synthetic",
           "config": {"workload": "isentropic vortex 200^2 periodic, R 20, Ma_v = 0.1 Ma, "
                                  "theta 240/1183, mu 1.5e-6, 50 convective times, "
                                  "Ma 0.3..1.3 x sigma 0..1 (+ original model at sigma 0)"},
           "map": summ, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_couette(args):
    """Thermal Couette flow (Sec. 4.4): the paper's 2 x 100 channel run to
    steady state in FP64 and FP32, with the error of the temperature profile
    against the closed form; then an 8192^2 FP32 channel with walls (linear
    shear, theta 0.2) timed against the same grid with periodic rows, which
    prices the wall pass."""
    import numpy as np
    import torch

    from paper_2002_03644_amd import Params, Solver, studies
    runs = {dt: studies.thermal_couette(ny=100, dtype=dt) for dt in ("f64", "f32")}
    n, thw, steps = args.n, 0.2, max(args.steps // 5, 20)
    eta = (np.arange(n, dtype=np.float64) / (n - 1))[:, None]
    fields = (np.ones((n, n)), 0.1 * eta * np.ones((1, n)), np.zeros((n, n)),
              np.full((n, n), thw))
    rate = {}
    for bc in ("wall", "periodic"):
        S = Solver(Params(n, n, dtype="f32", mu=1e-3, bc_y=bc, wall_ux_hi=0.1, wall_theta=thw,
                          theta_ref=thw), fields[0], fields[1], fields[2], theta=fields[3])
        S.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.step(steps)
        torch.cuda.synchronize()
        rate[bc] = n * n * steps / (time.perf_counter() - t0) / 1e6
        del S
        torch.cuda.empty_cache()
    r64 = runs["f64"]
    out = {"metric": "thermal Couette 2 x 100: steps per second to steady state (FP64)",
           "value": round(r64["steps"] / r64["seconds"], 1), "unit": "steps/s",
           "n_gpus": 1, "steps": r64["steps"], "warmup": 0,
           "ms_per_step": round(r64["seconds"] * 1e3 / r64["steps"], 5),
           "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "thermal Couette flow, 2 x 100 channel, Ma 0.8, Pr 0.71, "
                                  "gamma 1.4, sigma 0.9, T_w / T_r = 0.2, nu 0.1"},
           "couette": {dt: {"theta_error_vs_closed_form": r["error"],
                            "ux_error": r["ux_error"], "steps": r["steps"],
                            "seconds": round(r["seconds"], 3)} for dt, r in runs.items()},
           "walls_8192": {"mlups_walls": round(rate["wall"], 1),
                          "mlups_periodic": round(rate["periodic"], 1),
                          "steps": steps},
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def batch_cpu_baseline(specs, params, fields, count=12, steps=10, seed=0):
    """The FP64 oracle on a bounded sample of the batch: `count` domains
    drawn at random (seeded) from the batch, `steps` steps each after one
    warm-up step, on the host cores; MLUPS over the sample's node updates."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(seed)
    pick = sorted(rng.choice(len(specs), size=count, replace=False).tolist())
    nodes, secs = 0, 0.0
    for k in pick:
        p = params[k]
        r, u, v, t = fields[k]
        S = oracle.OracleSolver(oracle.OracleParams(p.nx, p.ny, mu=p.mu, sigma=p.sigma), r, u, v,
                                theta=t)
        S.step(1)
        t0 = time.perf_counter()
        S.step(steps)
        secs += time.perf_counter() - t0
        nodes += p.nx * p.ny * steps
        del S
    return {"value": round(nodes / secs / 1e6, 3), "unit": "MLUPS", "cores": oracle.threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{count} domains of the batch (indices {pick}, "
                      f"{sum(params[k].nx * params[k].ny for k in pick)} nodes), {steps} steps "
                      f"each after 1 warm-up step, FP64, {secs:.1f} s"}


def bench_batch(args):
    """256 independent periodic domains (sizes log-uniform 64..1016, vortex or
    turbulence, Mach 0.1-2.0, seed 0), FP32, graph-replayed persistent
    launches.  Domains whose flow leaves the method's stability range
    diverge and are frozen (their tiles are skipped); the value counts only
    the lattice updates actually performed.  The step at which each domain
    diverges is found in an untimed pass over the same steps (the run is
    deterministic: the timed run is checked to flag the same domains), and a
    domain counts its full steps inside the timed window; the step in which
    it is flagged, partly done, is left out (upper bound reported beside)."""
    import numpy as np
    import torch

    import hlbm_inputs as hi
    from paper_2002_03644_amd import BatchSolver, Params
    specs = hi.batch_specs(256, seed=0)
    params = [Params(sp.n, sp.n, dtype="f32", mu=1e-3, sigma=0.0, theta_ref=sp.theta,
                     steps_per_launch=args.steps_per_launch) for sp in specs]
    fields = [hi.batch_domain_fields(sp) for sp in specs]
    B = BatchSolver(params, fields)
    if args.tile_w and args.tile_h:
        B.set_tile(args.tile_w, args.tile_h, args.batch_kernel)
    else:
        B.autotune(steps=10)
    spl, bk, tw, th = B.plan()
    sizes = np.array([p.nx * p.ny for p in params], dtype=np.int64)
    W, K = args.warmup, args.steps
    # untimed pass over the same sequence of launches as the timed run (the
    # graphs replay the same kernels): spl-step launches, then one-step
    # launches for a remainder, for the warm-up and then the timed steps.
    # A domain flagged in the launch covering steps (a, b] did a steps in full.
    seq = [spl] * (W // spl) + [1] * (W % spl) + [spl] * (K // spl) + [1] * (K % spl)
    snap = B.save_state()
    never = np.iinfo(np.int64).max
    div = np.full(len(params), never, dtype=np.int64)   # steps done before the flagging launch
    div_end = np.full(len(params), never, dtype=np.int64)
    done_steps = 0
    for n_l in seq:
        B.step(n_l, graph=False)
        _, flags = B.status()
        new = (flags != 0) & (div == never)
        div[new] = done_steps
        div_end[new] = done_steps + n_l
        done_steps += n_l
    B.load_state(snap)          # same state, flags cleared
    del snap
    B.step(W, graph=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(B.stream)
    B.step(K, graph=True)
    e1.record(B.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    bad, flags = B.status()
    expect = div != never
    deterministic = bool(np.array_equal(flags != 0, expect))
    # full steps of each domain inside the window (W, W + K]; the flagging
    # launch (at most spl steps) is the partial part
    full = np.clip(np.minimum(div, W + K) - W, 0, K)
    partial = np.where(div != never,
                       np.clip(np.minimum(div_end, W + K) - np.maximum(div, W), 0, K), 0)
    done = int((sizes * full).sum())
    upper = int((sizes * (full + partial)).sum())
    mlups = done / (ms / 1e3) / 1e6
    gbs = BYTES_PER_NODE * done / (ms / 1e3) / 1e9
    cpu = None if args.no_cpu_baseline else batch_cpu_baseline(specs, params, fields)
    out = {"metric": "batched HLBM aggregate MLUPS (256 domains)", "value": round(mlups, 1),
           "unit": "MLUPS", "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": round(ms / K, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "256 periodic domains 64^2..1016^2 (seed 0), vortex or "
                                  "turbulence, Mach 0.1-2.0, FP32, hipGraph replay",
                      "nodes_total": int(sizes.sum()),
                      "node_updates_stated": int(sizes.sum()) * K,
                      "node_updates_performed": done,
                      "node_updates_upper_bound": upper,
                      "upper_bound_mlups": round(upper / (ms / 1e3) / 1e6, 1),
                      "domains_diverged_by_end": int(bad),
                      "domains_active_whole_window": int((div == never).sum()),
                      "divergence_steps_reproduced": deterministic,
                      "steps_per_launch": spl, "batch_kernel": bk, "tile_w": tw, "tile_h": th},
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "traffic": None,
                        "algorithmic_bytes": "80 B per performed lattice update"},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
