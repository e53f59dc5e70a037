"""Throughput benchmark: shifted solves per second on one MI355X.

Workload (default): n = 10^4, m = p = 8, 2000 imaginary-axis shifts
1j*logspace(-3, 3) on a random stable system (A = N(0, 1/n) - 1.5 I), the
configuration the headline metric is quoted on.  A step is one complete
solve of all shifts with the backward error of every shift certified:

  * FP64 form: FP64 sweep + Q* pass + G + FP64 residual/eta (value);
  * mixed form: FP32 sweep + FP64 refinement to eta <= 1e-13 (reported
    beside it in "mixed").

The one-time controller-Hessenberg reduction is timed separately.  Inputs
are resident in HBM before the timed region.  The JSON line also carries the
roofline of the dominant kernel (the one with the largest time per step among
the blocked sweep's update GEMM and tile kernel and the FP64 residual) and
the oracle timed on this host's cores on a bounded sample of shifts.

Beside the timed workload (not part of `value`): the serving mix (a closed
burst, then Poisson arrivals at 50% and 80% of the measured capacity, with
latency from arrival), and `other_workloads` at full size: n = 4096, m = 4,
1000 shifts and the n = 16384, m = 10 complex-plane grid (its structured
pseudospectrum included), each in both forms, and the interpolation method
at n = 15000, m = p = 10, r = 100 (`--no-extra` and `--serve-requests 0`
skip them).
"""
from __future__ import annotations

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

import workloads  # noqa: E402

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector and matrix (256 CU x 2.4 GHz x 128 flop/clk)
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector, published (packed FP32); issue without packing is half
HBM_PEAK_GBS = 8000.0


def sweep_flops(n: int, m: int) -> float:
    """Algorithmic flops of one structured sweep: (8m+2) n^2 real flops.

    Step k applies one reflector of size m+1 to the k rows above it: a
    complex dot product of length m+1 (m complex multiply-adds plus one add),
    a real-complex scaling and an m-term complex update, 16m+4 flops per row;
    summing k over the n steps gives (16m+4) n^2 / 2.
    """
    return (8.0 * m + 2.0) * n * n


def measured_traffic():
    """HBM bytes per launch of the solver kernels, from the rocprofv3
    FETCH_SIZE / WRITE_SIZE passes recorded in profiles/hbm_traffic.txt
    (scaled by a plain device copy of known size).  A kernel's figure is used
    only while its source file still hashes to the recorded value; otherwise
    the counters describe an older kernel and traffic is null."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return {}
    out = {}
    for name, k in rec.get("kernels", {}).items():
        try:
            sha = hashlib.sha256(open(os.path.join(ROOT, k["source"]), "rb").read()).hexdigest()
        except OSError:
            continue
        if sha == k.get("source_sha256"):
            out[name] = k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
    return out


def residual_flops(n: int, m: int) -> float:
    """FP64 residual H X - sigma X for one shift: real H (upper part + m
    subdiagonals, ~n^2/2 nonzeros) times 2m real columns, 2 flops each."""
    return 2.0 * (n * n / 2.0 + n * m) * 2.0 * m


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--mode", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle shifts (0 = automatic)")
    ap.add_argument("--scale", type=float, default=1.0, help="shrink n and s (smoke runs only)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests per load level in the serving leg (0 = skip the leg)")
    ap.add_argument("--serve-scale", type=float, default=1.0, help="scale n of the serving systems")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (n = 4096 FP64/mixed, the n = 16384 grid with its "
                         "pseudospectrum, the interpolation method)")
    ap.add_argument("--irka-iters", type=int, default=30)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 512 MiB once before the solves (a known-size kernel for HBM counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(shifts shard across GPUs with no collective in the hot loop, "
                                   "but multi-GPU runs are not part of it)"}))
        sys.exit(2)
    import torch

    import paper_1708_06290_amd as ss

    if args.serve_only:
        print(json.dumps({"serving": serving_leg(args)}))
        return
    wl = {"c1": workloads.C1, "c2": workloads.C2, "c3": workloads.C3, "c5": workloads.C5}[args.workload]
    n = max(wl.m + 1, int(wl.n * args.scale))
    s = max(1, int(wl.s * args.scale))
    m, p = wl.m, wl.p
    t0 = time.time()
    A, B, C = workloads.system(n, m, p, wl.seed)
    if wl.shifts_kind == "imag":
        shifts = workloads.imag_axis_shifts(wl.lo, wl.hi, s)
    else:
        shifts = workloads.plane_grid_shifts()[:s]
    print(f"# inputs generated in {time.time() - t0:.1f}s: n={n} m={m} p={p} s={s}", file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sysm = ss.System(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), torch.from_numpy(C).to(dev))
    info = sysm.info()
    print(f"# reduction {info['reduce_ms']:.1f} ms", file=sys.stderr, flush=True)
    del A
    dshifts = torch.from_numpy(shifts).to(dev)
    outputs = ss.SHS_OUT_X | ss.SHS_OUT_G | ss.SHS_OUT_ETA
    Xs = torch.empty((s * m, n), dtype=torch.complex128, device=dev)
    Gs = torch.empty((s * m, p), dtype=torch.complex128, device=dev)
    eta = torch.empty(s, dtype=torch.float64, device=dev)
    status = torch.empty(s, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        # a plain device copy of 512 MiB: its FETCH_SIZE / WRITE_SIZE readings
        # scale the counters of the solver kernels to bytes
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    results = {}
    modes = ["fp64", "mixed"] if args.mode == "both" else [args.mode]
    if "fp64" in modes:
        modes = ["fp64_uncertified"] + modes
    for mode_name in modes:
        mode = ss.SHS_MODE_FP32_REFINE if mode_name == "mixed" else ss.SHS_MODE_FP64
        # the uncertified FP64 form skips the residual GEMM and eta
        outs = (ss.SHS_OUT_X | ss.SHS_OUT_G) if mode_name == "fp64_uncertified" else outputs
        wbytes = sysm.workspace_bytes(s, mode, outs)
        work = torch.empty(wbytes, dtype=torch.uint8, device=dev)

        def step():
            ss.shs_solve(sysm.handle, dshifts, Xs, Gs, eta, status, mode=mode, outputs=outs,
                         tol=1e-13, max_iter=5, work=work, stream=stream)

        sysm.set_timing(False)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        sysm.set_timing(True)
        phase = {}
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        t1 = time.perf_counter()
        for (ea, eb) in evs:
            ea.record(stream)
            step()
            eb.record(stream)
            tm = sysm.last_timings()      # waits for this step's last event only
            for k, v in tm.items():
                phase[k] = phase.get(k, 0) + v
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        sysm.set_timing(False)
        step_ms = np.array([ea.elapsed_time(eb) for (ea, eb) in evs])
        e = eta.cpu().numpy()
        st = status.cpu().numpy()
        certified = mode_name != "fp64_uncertified"
        results[mode_name] = {
            "solves_per_s": s * args.steps / el,
            "ms_per_step": 1e3 * el / args.steps,
            # per-step device time (HIP events around each solve)
            "step_ms_median": round(float(np.median(step_ms)), 3),
            "step_ms_p99": round(float(np.percentile(step_ms, 99)), 3),
            "solves_per_s_median": round(s / (float(np.median(step_ms)) * 1e-3), 2),
            "eta_max": (float(np.nanmax(e)) if e.size else 0.0) if certified else None,
            "certified": bool((e <= 1e-13).all()) if certified else False,
            "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
            "phase_ms_per_step": {k: v / args.steps for k, v in phase.items() if k.endswith("_ms")},
            "launches_per_step": {k: v / args.steps for k, v in phase.items() if k.endswith("_calls")},
            "flops_per_step": {k: v / args.steps for k, v in phase.items() if k.endswith("_flops")},
            "shifts_per_step": {k: v / args.steps for k, v in phase.items() if k.endswith("_shifts")},
            "refine_iterations": phase.get("refine_iterations", 0) / args.steps,
            "fallback_shifts": phase.get("fallback_shifts", 0) / args.steps,
        }
        print(f"# {mode_name}: {results[mode_name]}", file=sys.stderr, flush=True)
        del work
        torch.cuda.empty_cache()

    # roofline of the dominant kernel (largest time per step) of the FP64
    # form, and of the other two big ones beside it.  Each kernel's time is
    # the sum of its launches, from HIP events on the solve stream.
    roof = None
    kernels = {}
    if "fp64" in results:
        r = results["fp64"]
        ph, calls = r["phase_ms_per_step"], r["launches_per_step"]
        # algorithmic flops of the launches the library made (per step)
        tile_f = r["flops_per_step"].get("sweep_tile_flops", 0.0)
        upd_f = r["flops_per_step"].get("sweep_update_flops", 0.0)
        # real columns per shift of the structured sweep (2m rounded up to a
        # power of two, or to 24 for 2m in 17 .. 24), the kernel's template width
        w = 2 if m <= 1 else 4 if m <= 2 else 8 if m <= 4 else 16 if m <= 8 else 24 if m <= 12 else 32
        cand = [
            (f"zupd_kernel<{w}>", "mfma", ph.get("sweep_update_ms", 0.0), calls.get("sweep_update_calls", 0), upd_f),
            (f"blk_tri_kernel<{m}>", "alu", ph.get("sweep_tile_ms", 0.0), calls.get("sweep_tile_calls", 0), tile_f),
            ("residual_mfma_kernel", "mfma", ph.get("residual_ms", 0.0), calls.get("residual_calls", 0),
             residual_flops(n, m) * s),
        ]
        traffic = measured_traffic()
        for name, bound, ms, nl, fl in cand:
            if ms <= 0 or nl <= 0:
                continue
            achieved = fl / (ms * 1e-3) / 1e12
            tb = traffic.get(name)
            # measured HBM bytes per launch over the average launch time,
            # against the 8 TB/s HBM peak
            gbs = None if tb is None else tb / (ms / nl * 1e-3) / 1e9
            kernels[name] = {"bound": bound, "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                             "traffic": None if tb is None else round(tb),
                             "hbm_gbs": None if gbs is None else round(gbs, 1),
                             "hbm_frac": None if gbs is None else round(gbs / HBM_PEAK_GBS, 4),
                             "ms_per_step": round(ms, 3), "launches_per_step": nl,
                             "avg_launch_ms": round(ms / nl, 4), "flops_per_launch": fl / nl}
        if kernels:
            top = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
            roof = {"kernel": top, **kernels[top]}
    # the mixed form's kernels: the blocked FP32 sweeps (FP32 tile kernels and
    # the all-shift update on the FP32 matrix cores, for the structured sweep
    # and for the dense-right-hand-side corrections) and the FP64 residuals.
    # The update's algorithmic flops per shift are the FP64 solve's (same
    # schedule, same tile height at this m), twice that for a correction
    # (4m instead of 2m real columns per shift).
    mixed_kernels = {}
    if "mixed" in results:
        r = results["mixed"]
        ph, calls = r["phase_ms_per_step"], r["launches_per_step"]
        # shift-solves of the correction sweeps; each also gets one more residual
        nd = r["shifts_per_step"].get("sweep32_dense_shifts", 0.0)
        upd_ps = (results["fp64"]["flops_per_step"].get("sweep_update_flops", 0.0) / s) if "fp64" in results else 0.0
        cand = [
            ("zupd32_kernel (structured + corrections)", "mfma", FP32_PEAK_TFLOPS, ph.get("sweep_update_ms", 0.0),
             calls.get("sweep_update_calls", 0), upd_ps * (s + 2.0 * nd)),
            ("residual_mfma_kernel", "mfma", FP64_PEAK_TFLOPS, ph.get("residual_ms", 0.0),
             calls.get("residual_calls", 0), residual_flops(n, m) * (s + nd)),
        ]
        for name, bound, peak, ms, nl, fl in cand:
            if ms <= 0 or nl <= 0 or fl <= 0:
                continue
            achieved = fl / (ms * 1e-3) / 1e12
            mixed_kernels[name] = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                                   "frac": round(achieved / peak, 4), "ms_per_step": round(ms, 3),
                                   "launches_per_step": nl}
        mixed_kernels["blk_tri_kernel<float> (structured + corrections)"] = {
            "bound": "alu", "ms_per_step": round(ph.get("sweep_tile_ms", 0.0), 3),
            "launches_per_step": calls.get("sweep_tile_calls", 0)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sysm, shifts, args.cpu_sample, n, m)
    del Xs, Gs
    sysm.close()
    torch.cuda.empty_cache()
    serving = serving_leg(args) if args.serve_requests > 0 else None
    extra = None
    if not args.no_extra:
        extra = {"c2": workload_leg(workloads.C2, ["fp64", "mixed"], 20, 3),
                 "c5": workload_leg(workloads.C5, ["fp64", "mixed"], 3, 1, pspec=True),
                 "irka": irka_leg(args.irka_iters) if args.irka_iters > 0 else None}

    head = results.get("fp64") or results.get("mixed")
    line = {
        "metric": "shifted solves/sec at n=1e4,m=8 (FP64 vs FP32+refine @1e-13 bwd err); p99",
        "value": round(head["solves_per_s"], 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if "fp64" in results else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name if args.scale == 1.0 else f"{wl.name}@scale{args.scale}",
                   "n": n, "m": m, "p": p, "shifts": s, "form": "fp64 sweep, eta certified",
                   "reduce_ms": round(info["reduce_ms"], 1)},
        "roofline": roof,
        "kernels": kernels,
        "mixed_kernels": mixed_kernels,
        "cpu_baseline": cpu,
        "fp64": results.get("fp64"),
        "fp64_uncertified": results.get("fp64_uncertified"),
        "mixed": results.get("mixed"),
        "serving": serving,
        "other_workloads": extra,
    }
    print(json.dumps(line))


def serving_leg(args):
    """Continuous-batching server over the eight resident systems of the
    serving mix (n in {1024..8192}, m in {1,2,4,16}, p = m): capacity from a
    closed burst, then Poisson arrivals at 50% and 80% of it; requests hold
    16..512 imaginary shifts, FP64 and mixed-precision interleaved."""
    import torch

    import paper_1708_06290_amd as ss
    t0 = time.time()
    systems = []
    for i in range(len(workloads.SERVE_SYSTEMS)):
        A, B, C = workloads.serve_system(i, args.serve_scale)
        systems.append(ss.System(A, B, C))
    red_ms = [round(sy.info()["reduce_ms"], 1) for sy in systems]
    print(f"# serving: {len(systems)} systems reduced in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    def run(reqs, rate_hz, label, keep=6):
        """Submit the stream; completed requests are checked (eta) and their
        outputs released as the stream goes, except the first `keep`, so
        long streams fit in device memory."""
        srv = ss.Server(streams=4, budget_bytes=64 << 30, max_batch=64)
        ids = [srv.register(sy) for sy in systems]
        kept, pending = [], []
        bad = 0

        def settle(h, block):
            nonlocal bad
            if block:
                srv.wait(h, timeout_ms=600000)
            elif srv.poll(h) < 2:
                return False
            e = h.eta.cpu().numpy() if h.eta is not None else None
            if e is not None and not (e <= 1e-13).all():
                bad += 1
            return True

        t_start = time.perf_counter()
        c_start = ss.shs_server_clock()
        for (t_arr, sys_id, shifts, mode) in reqs:
            if rate_hz is not None:
                delay = t_arr - (time.perf_counter() - t_start)
                if delay > 0:
                    time.sleep(delay)
            md = ss.SHS_MODE_FP64 if mode == "fp64" else ss.SHS_MODE_FP32_REFINE
            # latency runs from the scheduled arrival, so any lag of this
            # submitting loop counts against the server
            h = srv.submit(ids[sys_id], shifts, mode=md, arrival_s=c_start + t_arr if rate_hz is not None else 0.0)
            if len(kept) < keep:
                kept.append((h, sys_id, shifts, mode))
            pending.append(h)
            while pending and settle(pending[0], False):
                pending.pop(0)
        for h in pending:
            settle(h, True)
        for (h, _, _, _) in kept:
            srv.wait(h, timeout_ms=600000)
        el = time.perf_counter() - t_start
        st = srv.stats()
        handles = kept
        out = {"requests": len(reqs), "rate_hz": rate_hz, "wall_s": round(el, 3),
               "solves_per_s": round(st["solves"] / el, 2), "p50_ms": round(st["p50_ms"], 2),
               "p99_ms": round(st["p99_ms"], 2), "max_ms": round(st["max_ms"], 2),
               "latency_from": "arrival" if rate_hz is not None else "submit",
               "batches": st["batches"], "max_batch_systems": st["max_batch_systems"],
               "max_batch_requests": st["max_batch_requests"],
               "failed": st["failed"], "uncertified": bad}
        print(f"# serving {label}: {out}", file=sys.stderr, flush=True)
        return out, handles, srv, ids

    nreq = args.serve_requests
    # capacity from a closed burst of up to 1024 requests: the sustained rate
    # with the queue never empty (a short burst over-states it, its wall time
    # ending before the large requests' tail is paid)
    burst = workloads.request_stream(min(nreq, 1024), rate_hz=1e9, seed=workloads.ARRIVAL_SEED + 1)
    cal, _, srv, _ = run(burst, None, "burst")
    srv.close()
    cap = cal["requests"] / cal["wall_s"]
    levels = {}
    keep = None
    for frac in (0.5, 0.8):
        reqs = workloads.request_stream(nreq, rate_hz=frac * cap, seed=workloads.ARRIVAL_SEED)
        res, handles, srv, ids = run(reqs, frac * cap, f"{int(frac * 100)}%")
        levels[f"load_{int(frac * 100)}"] = res
        if keep is None:
            keep = (handles[:6], srv, ids)
        else:
            srv.close()
    # the same requests alone on the idle server: results must be bitwise
    # equal to the mix (both modes)
    handles, srv, ids = keep
    same = 0
    checked = 0
    for (h, sys_id, shifts, mode) in handles:
        md = ss.SHS_MODE_FP64 if mode == "fp64" else ss.SHS_MODE_FP32_REFINE
        alone = srv.wait(srv.submit(ids[sys_id], shifts, mode=md), timeout_ms=600000)
        torch.cuda.synchronize()
        checked += 1
        same += int(torch.equal(alone.X, h.X.t()))
    srv.close()
    for sy in systems:
        sy.close()
    return {"systems": [list(x) for x in workloads.SERVE_SYSTEMS], "n_scale": args.serve_scale,
            "reduce_ms": red_ms, "capacity_req_per_s": round(cap, 2), "burst": cal, **levels,
            "alone_vs_mix_bitwise": f"{same}/{checked}"}


def cpu_baseline(sysm, shifts, sample, n, m):
    """The oracle (plain C LU with partial pivoting, OpenMP over shifts) on a
    bounded sample of the same reduced systems, on this host's cores."""
    import oracle
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    threads = oracle.max_threads()
    if sample <= 0:
        # about 10-30 s of CPU work: O(n^2 m) per shift on the m-Hessenberg matrix
        per_shift_s = 4.0 * m * n * n / 1.5e9 + 1e-3
        sample = int(max(1, min(len(shifts), threads * max(1, round(15.0 / (per_shift_s * 1.0))))))
        sample = max(1, min(sample, 4 * threads, len(shifts)))
    idx = workloads.subset_indices(len(shifts), sample)
    t0 = time.perf_counter()
    oracle.solve(H, R, Ct, shifts[idx], nthreads=threads)
    el = time.perf_counter() - t0
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(len(idx) / el, 4), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": f"{len(idx)} of {len(shifts)} shifts (spread evenly), reduced system (H, R, Ct) "
                      f"from the GPU reduction, {el:.1f} s"}


def workload_leg(wl, modes, steps, warmup, pspec=False):
    """Another workload at full size: per-step device time (HIP events around
    each solve on the solve's stream) over `steps` repeats, every shift's
    backward error, and for the complex-plane grid the structured
    pseudospectrum ||G(z)||_2 of every point (shs_transfer_norm2)."""
    import torch

    import paper_1708_06290_amd as ss
    t0 = time.time()
    A, B, C = workloads.system(wl.n, wl.m, wl.p, wl.seed)
    shifts = wl.shifts()
    dev = torch.device("cuda", 0)
    sysm = ss.System(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), torch.from_numpy(C).to(dev))
    del A
    n, m, p, s = wl.n, wl.m, wl.p, wl.s
    out = {"n": n, "m": m, "p": p, "shifts": s, "reduce_ms": round(sysm.info()["reduce_ms"], 1)}
    dshifts = torch.from_numpy(shifts).to(dev)
    Xs = torch.empty((s * m, n), dtype=torch.complex128, device=dev)
    Gs = torch.empty((s * m, p), dtype=torch.complex128, device=dev)
    eta = torch.empty(s, dtype=torch.float64, device=dev)
    status = torch.empty(s, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    outs = ss.SHS_OUT_X | ss.SHS_OUT_G | ss.SHS_OUT_ETA
    for mode_name in modes:
        mode = ss.SHS_MODE_FP32_REFINE if mode_name == "mixed" else ss.SHS_MODE_FP64
        work = torch.empty(sysm.workspace_bytes(s, mode, outs), dtype=torch.uint8, device=dev)

        def step():
            ss.shs_solve(sysm.handle, dshifts, Xs, Gs, eta, status, mode=mode, outputs=outs, tol=1e-13,
                         max_iter=5, work=work, stream=stream)

        for _ in range(warmup):
            step()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for (ea, eb) in evs:
            ea.record(stream)
            step()
            eb.record(stream)
        torch.cuda.synchronize()
        ms = np.array([ea.elapsed_time(eb) for (ea, eb) in evs])
        e, st = eta.cpu().numpy(), status.cpu().numpy()
        out[mode_name] = {"steps": steps, "step_ms_median": round(float(np.median(ms)), 3),
                          "step_ms_p99": round(float(np.percentile(ms, 99)), 3),
                          "solves_per_s_median": round(s / (float(np.median(ms)) * 1e-3), 1),
                          "eta_max": float(np.nanmax(e)), "certified": bool((e <= 1e-13).all()),
                          "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))}}
        del work
        torch.cuda.empty_cache()
    if pspec:
        # structured pseudospectrum over the grid, from the last solve's G
        norms = torch.empty(s, dtype=torch.float64, device=dev)
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea.record(stream)
        ss.shs_transfer_norm2(Gs, m, norms, stream)
        eb.record(stream)
        torch.cuda.synchronize()
        nv = norms.cpu().numpy()
        out["pseudospectrum"] = {"points": s, "ms": round(ea.elapsed_time(eb), 3),
                                 "norm2_min": float(nv.min()), "norm2_max": float(nv.max()),
                                 "points_in_eps_0.01": int((nv >= 100.0).sum()),
                                 "points_in_eps_0.1": int((nv >= 10.0).sum())}
    sysm.close()
    del Xs, Gs
    torch.cuda.empty_cache()
    print(f"# {wl.name}: {out} ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    return out


def irka_leg(iters):
    """The interpolation method on a random system (n = 15000, m = p = 10,
    r = 100, the paper's Section 4.5 setting): every n-sized step on the GPU
    (per-shift-direction solves, transposed solves, projection), the r x r
    pencil on the host."""
    import torch

    import paper_1708_06290_amd as ss
    from paper_1708_06290_amd.irka import irka
    n, m, r = workloads.IRKA_N, workloads.IRKA_M, workloads.IRKA_R
    t0 = time.time()
    A, B, C = workloads.system(n, m, m, workloads.IRKA_SEED)
    dev = torch.device("cuda", 0)
    sysm = ss.System(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), torch.from_numpy(C).to(dev))
    del A
    red = sysm.info()["reduce_ms"]
    pts, bd, cd = workloads.irka_start(m, m, r, workloads.IRKA_SEED)
    irka(sysm, pts, bd, cd, iters=1)             # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = irka(sysm, pts, bd, cd, iters=iters)
    el = time.perf_counter() - t1
    last, prev = np.sort_complex(res.points[-1]), np.sort_complex(res.points[-2])
    out = {"n": n, "m": m, "p": m, "r": r, "iterations": iters, "reduce_ms": round(red, 1),
           "total_s": round(el, 3), "s_per_iteration": round(el / iters, 4),
           "solve_s": round(res.solve_s, 3), "project_s": round(res.project_s, 3), "host_s": round(res.host_s, 3),
           "shifted_solves_per_s": round(2 * r * iters / res.solve_s, 1), "max_eta": res.max_eta,
           "last_step_point_change": float(np.abs(last - prev).max() / np.abs(last).max())}
    sysm.close()
    torch.cuda.empty_cache()
    print(f"# irka: {out} ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    main()
