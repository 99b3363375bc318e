#!/usr/bin/env python3
"""Benchmark of P1 element-residual integration on one MI355X.

A step is one pass of the hot path over the 3D variable-coefficient Laplacian
workload (P1 tetrahedra, 2^20 elements from a jittered 64^3 cube grid, 4-point
degree-2 rule, kappa ~ U[0.5, 2] per quadrature point, u ~ U[-1, 1]):
fem_geometry (coordinates and connectivity to J^{-1}, det J) followed by
fem_integrate_residual, FP32. Inputs are resident in HBM before timing. The
inputs are replicated into several copies (> 512 MB in total) and the steps
rotate through them, so the 256 MB last-level cache cannot serve a step from
the previous one.

Prints ONE JSON line. Extra sections (not part of `value`): FP64, the other
physics, the adjoint, the batched launch, the achievable HBM bandwidth of a
plain copy kernel, and the FP64 CPU oracle on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import pathlib
import sys
import time

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "element-integration GF/s & elements/s (FP32, FP64); % of HBM roofline"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--copies", type=int, default=8, help="input copies the steps rotate through")
    p.add_argument("--quick", action="store_true", help="main step only (no extra sections, no CPU baseline)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    return p.parse_args()


class Timer:
    """HIP events around launches on torch's current stream (the stream the
    library launches on)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = []

    def start(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def stop(self, s):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.pairs.append((s, e))

    def mean_ms(self):
        return sum(s.elapsed_time(e) for s, e in self.pairs) / max(len(self.pairs), 1)

    def median_ms(self):
        v = sorted(s.elapsed_time(e) for s, e in self.pairs)
        return v[len(v) // 2] if v else 0.0


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update((ROOT / f).read_bytes())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "residual_lane": ["paper_1607_04245_amd/csrc/residual_lane.hip", "paper_1607_04245_amd/csrc/fem_device.hpp"],
    "geometry": ["paper_1607_04245_amd/csrc/geometry.hip", "paper_1607_04245_amd/csrc/fem_device.hpp"],
}


def measured_traffic(kernel_key, workload):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source; else None."""
    f = ROOT / "profiles" / "traffic.json"
    if not f.exists():
        return None
    try:
        data = json.loads(f.read_text())
        rec = data[f"{kernel_key}:{workload}"]
    except (KeyError, ValueError):
        return None
    if rec.get("source_hash") != source_hash(KERNEL_SOURCES[kernel_key]):
        return None
    return rec.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the element stream shards "
              "without communication, so N GPUs would each run this same single-GPU workload.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1607_04245_amd import api, meshgen as mg, model

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    props = torch.cuda.get_device_properties(dev)
    log(f"device {props.name} {getattr(props, 'gcnArchName', '')} CUs {props.multi_processor_count} "
        f"mem {props.total_memory / 2**30:.0f} GiB")

    def to_dev(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)

    # ---------------------------------------------------------- main step --
    t0 = time.time()
    wl = mg.config(2)
    n = wl.n_elem
    dim, phys, rule = wl.dim, wl.physics, wl.rule
    log(f"workload {wl.name}: {n} elements, {wl.n_vert} vertices (built in {time.time() - t0:.1f}s)")

    def make_copies(dt, copies):
        base = dict(coords=to_dev(wl.coords, torch.float64), conn=to_dev(wl.conn, torch.int32),
                    u=to_dev(wl.u, dt), coef=to_dev(wl.coef, dt))
        out = []
        for _ in range(copies):
            c = {k: v.clone() for k, v in base.items()}
            c["inv_j"] = torch.empty((dim * dim, n), dtype=dt, device=dev)
            c["det_j"] = torch.empty((n,), dtype=dt, device=dev)
            c["R"] = torch.empty_like(c["u"])
            out.append(c)
        return out

    def step(c, t_geo=None, t_int=None):
        s = t_geo.start() if t_geo else None
        api.fem_geometry(c["coords"], c["conn"], c["det_j"].dtype, inv_j=c["inv_j"], det_j=c["det_j"])
        if t_geo:
            t_geo.stop(s)
        s = t_int.start() if t_int else None
        api.fem_integrate_residual(dim, phys, rule, c["inv_j"], c["det_j"], c["u"], c["coef"], out=c["R"])
        if t_int:
            t_int.stop(s)

    def run_steps(dt, steps, warmup, copies):
        cs = make_copies(dt, copies)
        for i in range(warmup):
            step(cs[i % copies])
        torch.cuda.synchronize()
        tg, ti = Timer(torch), Timer(torch)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            step(cs[i % copies], tg, ti)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        del cs
        return wall, tg.mean_ms(), ti.mean_ms()

    word = 4
    wall, geo_ms, int_ms = run_steps(torch.float32, args.steps, args.warmup, args.copies)
    ms_per_step = 1e3 * wall / args.steps
    value = n * args.steps / wall
    log(f"FP32 step {ms_per_step:.4f} ms: geometry {geo_ms * 1e3:.1f} us, integrate {int_ms * 1e3:.1f} us")

    int_bytes = model.forward_bytes(dim, phys, rule, word) * n
    geo_bytes = model.geometry_bytes(dim, n, wl.n_vert, word) * n
    flops = model.model_flops(dim, phys, rule)
    kernels = {
        "fem_integrate_residual": dict(avg_us=int_ms * 1e3, bytes=int_bytes,
                                       gbs=int_bytes / (int_ms * 1e-3) / 1e9,
                                       elements_per_s=n / (int_ms * 1e-3),
                                       model_gflops=n * flops / (int_ms * 1e-3) / 1e9),
        "fem_geometry": dict(avg_us=geo_ms * 1e3, bytes=geo_bytes, gbs=geo_bytes / (geo_ms * 1e-3) / 1e9,
                             elements_per_s=n / (geo_ms * 1e-3)),
    }
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"])
    dk = kernels[dom]
    kkey = "residual_lane" if dom == "fem_integrate_residual" else "geometry"
    traffic = measured_traffic(kkey, "laplace3d_2p20_f32")
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": dk["bytes"]}

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D variable-coefficient Laplacian, P1 tetrahedra, 2^20 elements of a jittered "
                               "64^3 Kuhn grid, 4-point degree-2 rule; step = fem_geometry + "
                               "fem_integrate_residual",
                   "n_elem": n, "n_vert": wl.n_vert, "copies": args.copies},
        "model_gflops": value * flops / 1e9,
        "kernels": kernels,
        "roofline": roofline,
    }

    if not args.quick:
        extra = {}
        # FP64 step
        wall64, g64, i64 = run_steps(torch.float64, max(10, args.steps // 2), 2, args.copies)
        b64 = model.forward_bytes(dim, phys, rule, 8) * n
        extra["fp64_step"] = dict(elements_per_s=n * max(10, args.steps // 2) / wall64,
                                  integrate_us=i64 * 1e3, integrate_gbs=b64 / (i64 * 1e-3) / 1e9,
                                  integrate_model_gflops=n * flops / (i64 * 1e-3) / 1e9, geometry_us=g64 * 1e3)
        log(f"FP64 integrate {i64 * 1e3:.1f} us ({extra['fp64_step']['integrate_gbs']:.0f} GB/s)")
        # achievable HBM bandwidth: copy of 2 GiB
        nb = 2 << 30
        src = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            api.fem_stream_copy(src, dst)
        tm = Timer(torch)
        for _ in range(10):
            s = tm.start()
            api.fem_stream_copy(src, dst)
            tm.stop(s)
        torch.cuda.synchronize()
        copy_gbs = 2 * nb / (tm.median_ms() * 1e-3) / 1e9
        extra["stream_copy"] = dict(bytes=2 * nb, median_us=tm.median_ms() * 1e3, gbs=copy_gbs)
        del src, dst
        roofline["frac_of_achievable"] = dk["gbs"] / copy_gbs
        log(f"stream copy {copy_gbs:.0f} GB/s")
        result["extra"] = extra

    if not args.quick and not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(wl, flops)

    print(json.dumps(result), flush=True)


def cpu_baseline(wl, flops):
    """The FP64 oracle (plain C, one thread) on the same step: geometry and
    residual of the first elements of the workload, repeated until about 10 s
    of CPU work has run."""
    import numpy as np

    import oracle

    sample = wl.n_elem
    reps, t_total = 0, 0.0
    while t_total < 10.0 and reps < 50:
        t = time.perf_counter()
        R, nd = oracle.residual(wl.dim, wl.physics, wl.rule, wl.coords, wl.conn, wl.u, wl.coef)
        t_total += time.perf_counter() - t
        reps += 1
    assert nd == 0 and np.isfinite(R).all()
    eps = sample * reps / t_total
    log(f"CPU oracle: {eps:.3e} elements/s over {reps} passes ({t_total:.1f} s)")
    return {"value": eps, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} passes of fem_oracle_residual (FP64 geometry + residual) over all {sample} "
                      f"elements of the step workload, {t_total:.1f} s single-threaded",
            "model_gflops": eps * flops / 1e9, "host_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()
