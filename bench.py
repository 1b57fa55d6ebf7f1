"""Benchmark of the coupled D3Q19 + IBM + FE swimmer step on one MI355X.

Workload: the single-swimmer 128^3 case (tau 0.8, Guo forcing, 4-point IBM
kernel, radius-4 beads with 1280 triangles, seeded phase and jitter).  A step
is one full pass of the hot path: bead statistics, membrane + driving + spring
forces, spreading, fused stream-collide, interpolation and advection.

Prints one JSON line: whole-step MLUPS (value), the stream-collide kernel's
achieved HBM bandwidth against the 8 TB/s peak (roofline), and the FP64 CPU
oracle timed on a bounded sample of the same workload (cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# stream-collide launch shapes (block, XCD remap, resident workgroups per CU),
# measured best for these workloads on MI355X by explicit sweeps: the 128^3
# FP32 step with one resident 512-node workgroup per CU claiming blocks in
# round-robin order (62.3 us against 63.0 us for two of 256 nodes, 64.9 us
# remapped); FP16 (static persistent walk) at two of 256 nodes; the batch
# and the 1024x256x256 box non-persistent with the XCD remap (batch 724.7
# against 729.5 us in block order, 760-940 us persistent; box 1.842 ms
# against 1.849 ms in block order and 1.869 ms at block 256).  The batch
# section itself runs the launch tuner (lbmib.tune_launch) and times the
# shape it picks (block order, 707.6 us against 731.5 us remapped, in the
# tuner's first run); BATCH_LAUNCH is that shape, which the parity test of
# the full ensemble uses.  The paper-box section tunes too.
MAIN_LAUNCH = (512, False, 1)
# The 128^3 workload's populations: FP32 deviations in one set updated in
# place (LBM_FP32_INPLACE; 159 MB instead of two sets of 319 MB, which the
# 256 MB last-level cache holds: step 56.6 against 57.6-58.5 us with two sets,
# bit-identical results)
MAIN_STORAGE = 3
FP16_LAUNCH = (256, False, 2)
BATCH_LAUNCH = (512, False, 0)
BOX_LAUNCH = (512, True, 0)
KERNEL_LAUNCH = (256, False, -1)  # serial order: full-grid launch for the roofline
PMC_PROFILE = os.path.join(ROOT, "profiles", "stream_collide_128cubed_pmc.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2202_12147_amd", "csrc", "lattice_kernels.hip")


def measured_traffic():
    """HBM bytes per full-grid stream-collide launch from the committed
    rocprofv3 counter runs, or None when the kernel source has changed since."""
    import hashlib
    try:
        fields = dict(line.split(": ", 1) for line in open(PMC_PROFILE).read().splitlines()
                      if line and not line.startswith("#"))
        src = open(KERNEL_SOURCE).read()
    except OSError:
        return None
    dev = src[:src.index("}  // namespace")]
    if hashlib.sha256(dev.encode()).hexdigest() != fields.get("kernel_source_sha256", "").strip():
        return None
    return int(fields["traffic_bytes_per_launch"])


def cpu_baseline(case, budget_s=12.0, single_budget_s=4.0):
    """Time the FP64 oracle on the same 128^3 workload for a few steps, on all
    allowed host cores (at most 16) and on one."""
    from oracle import orc
    cores = min(len(os.sched_getaffinity(0)), 16)
    nodes = case["shape"][0] * case["shape"][1] * case["shape"][2]

    def timed(threads, budget):
        orc.set_threads(threads)
        o = orc.Oracle(case["shape"], case["tau"], case["forcing"], case["width"])
        for sw in case["swimmers"]:
            o.add_swimmer_desc(sw)
        o.step(1)  # first touch
        steps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget:
            o.step(1)
            steps += 1
        return steps, time.perf_counter() - t0

    steps, dt = timed(cores, budget_s)
    s1, dt1 = timed(1, single_budget_s)
    model = ""
    try:
        model = next(line.split(":", 1)[1].strip() for line in open("/proc/cpuinfo")
                     if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{steps} FP64 steps of the same 128^3 swimmer workload (IBM included)",
            "single_thread_value": nodes * s1 / dt1 / 1e6, "single_thread_sample": f"{s1} steps",
            "cpu_model": model, "comparison": "FP64 CPU oracle vs FP32 GPU"}


def fp16_section(lbmib, wl, case, steps, warmup, gmax):
    """FP16-shifted storage on the same workload and GPU: throughput, kernel
    bandwidth (76 B per node), and the small case's swimmer displacement
    against the FP32 run on the same GPU (FP32 itself is pinned to the FP64
    oracle by the tests)."""
    import numpy as np
    S = lbmib.fp16_scale_for(gmax)
    nodes = case["shape"][0] * case["shape"][1] * case["shape"][2]
    lat = lbmib.from_workload(case, storage=lbmib.FP16_SHIFTED, fp16_scale=S)
    lat.set_stream_collide_launch(*FP16_LAUNCH)
    lat.step(warmup)
    lat.sync()
    t0 = time.perf_counter()
    lat.step(steps)
    lat.sync()
    dt = time.perf_counter() - t0
    lat.set_stream_collide_launch(*KERNEL_LAUNCH)
    lat.step(20)
    lat.set_kernel_timing(True)
    lat.step(min(steps, 2000))
    kms, n = lat.kernel_time()
    lat.set_kernel_timing(False)
    lat.sync()
    gbs = lat.bytes_per_step / (kms / n * 1e-3) / 1e9
    small = wl.small_case()
    disp = {}
    for name, st, sc in (("fp32", lbmib.FP32_SHIFTED, 1.0), ("fp16", lbmib.FP16_SHIFTED, 2.0 ** 27),
                         ("fp32_plain", lbmib.FP32_PLAIN, 1.0)):
        g = lbmib.from_workload(small, storage=st, fp16_scale=sc)
        x0 = g.swimmer_centres()[0, 0]
        g.step(small["steps"])
        disp[name] = g.swimmer_centres()[0, 0] - x0
    return {"storage": f"fp16 shifted, S=2^{int(np.log2(S))}", "value": round(nodes * steps / dt / 1e6, 1),
            "unit": "MLUPS", "ms_per_step": round(dt / steps * 1e3, 5),
            "kernel_gbs": round(gbs, 1), "kernel_frac": round(gbs / PEAK_HBM_GBS, 4),
            "bytes_per_launch": lat.bytes_per_step,
            "small_case_displacement": {"fp32": disp["fp32"], "fp16": disp["fp16"],
                                        "rel_diff": abs(disp["fp16"] - disp["fp32"]) / abs(disp["fp32"]),
                                        "fp32_plain": disp["fp32_plain"],
                                        "plain_rel_diff": abs(disp["fp32_plain"] - disp["fp32"]) / abs(disp["fp32"])}}


def average_section(lbmib, lat, nodes, steps=2000):
    """Cost of the time-averaged velocity field on the same handle: step
    time with every step sampled and with every tenth, and the full-grid
    stream-collide kernel of a sampled step, whose algorithmic traffic is
    152 + 48 bytes per node (the FP64 sums of u are read and written)."""
    res = {}
    for every in (1, 10):
        lat.average_begin(every)
        lat.step(64)
        lat.sync()
        t0 = time.perf_counter()
        lat.step(steps)
        lat.sync()
        res[f"every_{every}_ms_per_step"] = round((time.perf_counter() - t0) / steps * 1e3, 5)
    lat.average_begin(1)
    lat.set_stream_collide_launch(*KERNEL_LAUNCH)
    lat.step(20)
    lat.set_kernel_timing(True)
    lat.step(steps)
    kms, n = lat.kernel_time()
    lat.set_kernel_timing(False)
    lat.sync()
    lat.average_begin(0)
    lat.set_stream_collide_launch(*MAIN_LAUNCH)
    avg_ms = kms / max(n, 1)
    nbytes = lat.bytes_per_step + 48 * nodes
    res.update(sampled_kernel_ms=round(avg_ms, 5), bytes_per_sampled_launch=nbytes,
               sampled_kernel_gbs=round(nbytes / (avg_ms * 1e-3) / 1e9, 1))
    return res


def seeds_section(lbmib, wl, seeds=(1, 2), steps=4000, warmup=200):
    """The 128^3 workload drawn with other seeds (phase offset, radius and
    rest-length jitter) at the same launch shape: MLUPS per seed."""
    out = {}
    for seed in seeds:
        case = wl.single_128(seed=seed)
        nodes = case["shape"][0] * case["shape"][1] * case["shape"][2]
        lat = lbmib.from_workload(case, storage=MAIN_STORAGE)
        lat.set_stream_collide_launch(*MAIN_LAUNCH)
        lat.step(warmup)
        lat.sync()
        t0 = time.perf_counter()
        lat.step(steps)
        lat.sync()
        out[str(seed)] = round(nodes * steps / (time.perf_counter() - t0) / 1e6, 1)
        lat.close()
    return {"unit": "MLUPS", "steps": steps, "value_by_seed": out}


def batch_section(lbmib, wl, steps=5000, warmup=200, seed=0):
    """The 64-box ensemble (edges from {48,64,80,96} per axis, one swimmer
    each) advanced together at the launch shape the tuner picks for it
    (lbmib.tune_launch: every candidate timed on a scratch batch of the same
    ensemble, 200 steps, best of two passes), `steps` timed steps; batch
    MLUPS = total nodes x steps / time."""
    ens = wl.ensemble(seed=seed)
    t0 = time.perf_counter()
    best, table = lbmib.tune_launch(lambda: lbmib.batch_from_ensemble(ens))
    tune_s = time.perf_counter() - t0
    batch = lbmib.batch_from_ensemble(ens)
    batch.set_stream_collide_launch(*best)
    batch.step(warmup)
    batch.sync()
    t0 = time.perf_counter()
    batch.step(steps)
    batch.sync()
    dt = time.perf_counter() - t0
    return {"value": round(batch.N * steps / dt / 1e6, 1), "unit": "MLUPS", "steps": steps,
            "ms_per_step": round(dt / steps * 1e3, 4), "boxes": len(ens["boxes"]), "nodes": batch.N,
            "markers": batch.n_markers, "seed": seed,
            "launch": {"block": best[0], "xcd_remap": int(best[1]), "resident": best[2]},
            "tuner": {"seconds": round(tune_s, 1),
                      "us_per_step": {f"{b}/{int(r)}/{p}": round(v, 1) for (b, r, p), v in table.items()}}}


def adjoint_section(lbmib, wl, use_graphs=True):
    """Gradient of a swimmer's displacement over one 2000-step period on the
    96^3 adjoint workload (checkpoints every 100 steps): wall time of
    lbm_adjoint (checkpointed forward + segment recompute + reverse sweep)
    against the plain forward run of the same steps.  use_graphs=False
    launches every kernel directly (counter collection: the profiler's
    counter mode does not survive replays of the two-stream graphs)."""
    case = wl.adjoint_case(reduced=False)
    T, K = case["steps"], case["checkpoint"]
    nodes = case["shape"][0] * case["shape"][1] * case["shape"][2]
    lat = lbmib.from_workload(case, use_graphs=use_graphs)
    lat.step(200)
    lat.sync()
    t0 = time.perf_counter()
    lat.step(T)
    lat.sync()
    t_fwd = time.perf_counter() - t0
    lat.adjoint(T, K, rewind=True)  # workspace allocation, first launches
    t0 = time.perf_counter()
    J, grad = lat.adjoint(T, K, rewind=True)
    t_adj = time.perf_counter() - t0
    return {"workload": f"adjoint {case['shape'][0]}^3, one swimmer, T={T} steps, checkpoint {K}",
            "forward_ms": round(t_fwd * 1e3, 2), "adjoint_ms": round(t_adj * 1e3, 2),
            "ratio": round(t_adj / t_fwd, 3),
            "note": "adjoint_ms includes its own checkpointed forward run",
            "adjoint_mlups": round(nodes * T / t_adj / 1e6, 1),
            "J": J, "grad_A_B_alpha_k": [float(g) for g in grad]}


def paper_box_section(lbmib, wl, steps=500, warmup=50):
    """Throughput on the paper's 1024x256x256 box (67.1 M nodes, 10.2 GB of
    FP32 populations per step) with one radius-5 swimmer, at the launch shape
    the tuner picks on a scratch handle of the same box (60 steps per
    candidate, best of two passes)."""
    case = wl.paper_box()
    nodes = case["shape"][0] * case["shape"][1] * case["shape"][2]
    t0 = time.perf_counter()
    best, table = lbmib.tune_launch(lambda: lbmib.from_workload(case), steps=60, warmup=20)
    tune_s = time.perf_counter() - t0
    lat = lbmib.from_workload(case)
    lat.set_stream_collide_launch(*best)
    lat.step(warmup)
    lat.sync()
    t0 = time.perf_counter()
    lat.step(steps)
    lat.sync()
    dt = time.perf_counter() - t0
    return {"workload": case["name"], "nodes": nodes, "markers": lat.n_markers, "steps": steps,
            "value": round(nodes * steps / dt / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(dt / steps * 1e3, 4),
            "step_gbs": round(lat.bytes_per_step / (dt / steps) / 1e9, 1),
            "launch": {"block": best[0], "xcd_remap": int(best[1]), "resident": best[2]},
            "tuner": {"seconds": round(tune_s, 1),
                      "us_per_step": {f"{b}/{int(r)}/{p}": round(v, 1) for (b, r, p), v in table.items()}}}


def kernels_section(lbmib):
    """Full-grid stream-collide launches alone (serial launch mode, no
    swimmer), FP32 (two sets, and one set in place) and FP16-shifted
    storage, at 128^3 (populations of the
    order of the 256 MB last-level cache, which serves part of the traffic)
    and at 256^3 (2.55 GB FP32, 1.27 GB FP16: HBM only): mean launch
    duration from HIP events stamped by the dispatch packets, algorithmic
    bytes (19 loads + 19 stores per node) per second against the 8 TB/s peak.
    Each grid is timed twice on the same flow: with a uniform body force
    (every node carries the Guo source term) and, keys ending in `_f0`, after
    the force is switched off (as in the bulk of the swimmer workloads, where
    the source term is skipped)."""
    out = {}
    for name, edge, storage in (("fp32_128", 128, lbmib.FP32_SHIFTED), ("fp16_128", 128, lbmib.FP16_SHIFTED),
                                ("fp32_256", 256, lbmib.FP32_SHIFTED), ("fp16_256", 256, lbmib.FP16_SHIFTED),
                                ("fp32inplace_128", 128, lbmib.FP32_INPLACE),
                                ("fp32inplace_256", 256, lbmib.FP32_INPLACE)):
        lat = lbmib.Lattice((edge, edge, edge), 0.8, storage=storage, width=4, fp16_scale=2.0 ** 20)
        lat.set_body_force((1e-6, 0.0, 0.0))
        lat.set_stream_collide_launch(*KERNEL_LAUNCH)
        lat.step(20)
        for key, force in ((name, (1e-6, 0.0, 0.0)), (name + "_f0", (0.0, 0.0, 0.0))):
            lat.set_body_force(force)
            lat.step(2)
            lat.set_kernel_timing(True)
            lat.step(200)
            kms, n = lat.kernel_time()
            lat.set_kernel_timing(False)
            lat.sync()
            ms = kms / max(n, 1)
            gbs = lat.bytes_per_step / (ms * 1e-3) / 1e9
            out[key] = {"grid": [edge] * 3, "bytes_per_launch": lat.bytes_per_step, "avg_kernel_ms": round(ms, 5),
                        "gbs": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4), "launches": n,
                        "body_force": force[0]}
        lat.close()
    return out


def paper_length_section(lbmib, wl, periods, out_dir=None, arrangement=None, distance=None, v_ref=None,
                         tau=1.0):
    """The paper's runs over `periods` actuation periods of 2e4 steps on the
    1024x256x256 box (workloads.paper_run): one swimmer, or a pair one behind
    the other / side by side at a given distance of their middle beads.  Per
    period and swimmer the centre velocity (Eq. vel_swim); the Reynolds
    numbers of the swimmer (v_cm * 2 L / nu) and of the fastest bead (largest
    bead speed over the last period * 2 a / nu); with v_ref (a single
    swimmer's velocity) the relative change of each swimmer's velocity over
    the last period (Eq. inc); and the velocity field averaged over the last
    period (Figs. 3, 6, 9), saved downsampled when out_dir is set."""
    import numpy as np
    case = wl.paper_run(arrangement, distance, tau)
    sw = case["swimmers"][0]
    T = int(case["period"])
    nu = (case["tau"] - 0.5) / 3.0
    lat = lbmib.from_workload(case)
    lat.set_stream_collide_launch(*BOX_LAUNCH)
    X = [lat.swimmer_centres().copy()]
    per_period, bead_speed = [], 0.0
    t0 = time.perf_counter()
    chunk = 500
    for p in range(periods):
        last = p == periods - 1
        if last:
            lat.average_begin(1)
        R_prev = lat.bead_centres()
        for _ in range(T // chunk):
            lat.step(chunk)
            if last:
                R = lat.bead_centres()
                bead_speed = max(bead_speed, float(np.abs(R - R_prev).max()) / chunk)
                R_prev = R
        X.append(lat.swimmer_centres().copy())
        v = (X[-1] - X[-2]) / T  # [swimmer, 3]
        per_period.append(v)
        print(f"paper run: period {p + 1}/{periods}: v_cm " + " ".join(f"{vs[0]:.6e}" for vs in v) +
              f" l.u./step ({time.perf_counter() - t0:.0f} s)", flush=True)
    avg, count = lat.average_velocity()
    lat.average_begin(0)
    L = 2.0 * float(sw["L0"][0])
    a = float(sw["radius"][0])
    v_last = per_period[-1][:, 0]
    res = {"workload": case["name"], "periods": periods, "period_steps": T,
           "forcing": "shan-chen", "tau": case["tau"], "nu": nu,
           "swimmer_x0": [float(x[0]) for x in X[0]],
           "v_cm_per_period": [[float(vs[0]) for vs in v] for v in per_period],
           "v_cm_yz_last": [[float(c) for c in vs[1:]] for vs in per_period[-1]],
           "v_last": [float(x) for x in v_last], "Re_swim": float(np.abs(v_last).max()) * L / nu,
           "bead_speed_max_last_period": bead_speed, "Re_bead": bead_speed * 2.0 * a / nu,
           "mean_field_samples": count, "mean_field_max_abs": float(np.abs(avg).max()),
           "seconds": round(time.perf_counter() - t0, 1)}
    if arrangement is None:
        res["v_ref"] = float(v_last[0])
    if v_ref:
        res["v_delta_last"] = [float((v - v_ref) / v_ref) for v in v_last]
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        tag = "paper_run" if arrangement is None else f"paper_pair_{arrangement}_{distance:g}"
        np.save(os.path.join(out_dir, f"{tag}_mean_u_sub4.npy"), avg[:, ::4, ::4, ::4].astype(np.float32))
        np.save(os.path.join(out_dir, f"{tag}_mean_u_midplane.npy"), avg[:, avg.shape[1] // 2].astype(np.float32))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint section (profiling of the reverse sweep)")
    ap.add_argument("--direct", action="store_true",
                    help="with --adjoint-only: launch kernels directly, no graph replays (counter runs)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the full-grid stream-collide launches at 128^3 and 256^3 (counter runs)")
    ap.add_argument("--paper-length", type=int, default=0, metavar="PERIODS",
                    help="only the paper's single-swimmer run over PERIODS periods of 2e4 steps")
    ap.add_argument("--paper-out", default=None, help="directory for the paper run's averaged field")
    ap.add_argument("--paper-pair", default=None, choices=["collinear", "side"],
                    help="with --paper-length: two swimmers one behind the other or side by side")
    ap.add_argument("--paper-distance", type=float, default=144.0,
                    help="with --paper-pair: distance of the middle beads (lattice units)")
    ap.add_argument("--paper-vref", type=float, default=None,
                    help="with --paper-pair: a single swimmer's velocity, for the relative changes")
    ap.add_argument("--paper-tau", type=float, default=1.0,
                    help="with --paper-length: relaxation time (viscosity sweeps; the paper's run is 1)")
    ap.add_argument("--main-only", action="store_true",
                    help="skip the fp16, batch, adjoint and paper-box sections (counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2202_12147_amd import lbmib, workloads as wl

    torch.cuda.set_device(0)
    if args.adjoint_only:
        out = {"adjoint": adjoint_section(lbmib, wl, use_graphs=not args.direct)}
        if args.direct:  # the copy probe calibrates the byte counters of the same run
            out["copy_probe_gbs"] = lbmib.copy_bandwidth(1 << 30, 20)
        print(json.dumps(out), flush=True)
        return
    if args.kernels_only:
        print(json.dumps({"kernels": kernels_section(lbmib), "copy_probe_gbs": lbmib.copy_bandwidth(1 << 30, 20)}),
              flush=True)
        return
    if args.paper_length:
        print(json.dumps({"paper_length": paper_length_section(
            lbmib, wl, args.paper_length, args.paper_out, args.paper_pair,
            args.paper_distance if args.paper_pair else None, args.paper_vref, args.paper_tau)}), flush=True)
        return
    case = wl.single_128(seed=0)
    nodes = case["shape"][0] * case["shape"][1] * case["shape"][2]
    stream = torch.cuda.Stream()
    lat = lbmib.from_workload(case, storage=MAIN_STORAGE, stream=stream)
    lat.set_stream_collide_launch(*MAIN_LAUNCH)

    lat.step(args.warmup)
    lat.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(args.steps)
    torch.cuda.synchronize()  # the whole device: the library's side stream included
    dt = time.perf_counter() - t0
    lat.sync()  # then the overflow check (a bead outgrowing its tiles), outside the timed steps
    ms_per_step = dt / args.steps * 1e3
    value = nodes * args.steps / dt / 1e6

    # Roofline of the dominant kernel: the full-grid stream-collide launch,
    # timed with HIP events on the library stream while steps run in serial
    # order (immersed-boundary kernels, then one full-grid launch), so the
    # kernel has the device to itself and its duration is well defined.
    ksteps = min(args.steps, 2000)
    lat.set_stream_collide_launch(*KERNEL_LAUNCH)
    lat.step(50)
    lat.set_kernel_timing(True)
    lat.step(ksteps)
    kms, launches = lat.kernel_time()
    lat.set_kernel_timing(False)
    lat.sync()
    avg_ms = kms / max(launches, 1)
    achieved = lat.bytes_per_step / (avg_ms * 1e-3) / 1e9
    copy_gbs = lbmib.copy_bandwidth(1 << 30, 20)
    tbytes = measured_traffic()
    traffic = None if tbytes is None else round(tbytes / (avg_ms * 1e-3) / 1e9, 1)

    out = {
        "metric": "MLUPS & HBM GB/s of D3Q19+IBM step; adjoint/forward time ratio; batch MLUPS",
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single swimmer 128^3 (D3Q19 BGK Guo, tau 0.8, 4-point IBM, "
                               "3 beads r=4 x 1280 triangles, spacing 16, A=5e-4, T=2000)",
                   "grid": list(case["shape"]), "markers": lat.n_markers, "seed": 0,
                   "storage": "fp32 shifted, one set in place",
                   "launch": {"block": MAIN_LAUNCH[0], "xcd_remap": int(MAIN_LAUNCH[1]),
                              "resident": MAIN_LAUNCH[2]}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "traffic_bytes_per_launch": tbytes,
                     "kernel": "k_stream_collide<fp32 in place,256,all> (full grid, 19 loads + 19 stores per node)",
                     "avg_kernel_ms": round(avg_ms, 5), "launches_timed": launches,
                     "bytes_per_launch": lat.bytes_per_step,
                     "copy_probe_gbs": round(copy_gbs, 1),
                     "frac_of_copy_probe": round(achieved / copy_gbs, 4)},
    }
    lat.set_stream_collide_launch(*MAIN_LAUNCH)
    if not args.main_only:
        import numpy as np
        gmax = float(np.abs(lat.populations()).max())
        out["kernels"] = kernels_section(lbmib)
        out["average"] = average_section(lbmib, lat, nodes)
        out["seeds"] = seeds_section(lbmib, wl)
        out["fp16"] = fp16_section(lbmib, wl, case, args.steps, args.warmup, gmax)
        del lat
        out["batch"] = batch_section(lbmib, wl)
        out["adjoint"] = adjoint_section(lbmib, wl)
        out["paper_box"] = paper_box_section(lbmib, wl)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
