#!/usr/bin/env python3
"""Benchmark of P1 element-residual integration on one MI355X.

A step is one pass of the hot path over the 3D variable-coefficient Laplacian
workload (P1 tetrahedra, 2^20 elements of a jittered 64^3 Kuhn grid, 4-point
degree-2 rule, kappa ~ U[0.5, 2] per quadrature point, u ~ U[-1, 1]): element
residuals from coordinates, connectivity, closure and coefficients, in FP32,
with geometry and integration fused in one kernel
(fem_integrate_residual_mesh). The same step as two calls (fem_geometry, then
fem_integrate_residual) is reported beside it. All inputs are resident in HBM before the
timed region. They are replicated into at least 8 copies (> 600 MB of the
fused kernel's bytes in total) and the steps rotate through them, so the
256 MB last-level cache cannot serve a step from the data of the one before.

The timed region is one replay of a HIP graph holding the `--steps` steps
(captured with torch's graph capture on the stream the library launches on),
bracketed by one pair of HIP events; launching through Python one call at a
time would otherwise cost more host time than a step takes on the GPU.
Before it come the `--warmup` steps and then replays of the same graph until
the GPU has been busy for 0.1 s, so that the timed steps run at the clocks of
a loaded GPU (the first milliseconds after the host work between sections
run slower); every section is timed this way.

Prints ONE compact JSON line, last on stdout and below 4 KB (a few progress
lines go to stderr; --verbose prints one per section). `value` is elements
per second of the step (wall clock around the replay). The roofline object is
for the step's kernel, its duration being the events' elapsed time over the
replay divided by the number of launches in it. The line also summarises the
FP64 step, the integrate-only kernel (the paper's form, geometry precomputed),
the batched launch against the same 64 launches recorded in one graph, the
thread transposition against the lane kernel, and the FP64 CPU oracle. The
full record, with every extra section (elasticity, coefficient spaces,
gather form, mesh plans, P2/P3, element matrices, assembly, adjoint), is
written to gpurun_out/bench_extra.json (--extra-out).

Every timed section rotates through copies of its inputs sized on the bytes
its own kernel touches per launch: at least 8 copies and more than 600 MB in
total (2 copies when one launch alone moves more than that).
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
ROTATE_BYTES = 600e6  # rotate through input copies totalling at least this much
MIN_COPIES = 8       # and through at least this many copies
MAX_LINE = 4000      # the JSON line on stdout stays below this many bytes
PREHEAT_S = 0.1      # each timed section first keeps the GPU busy this long (untimed)


VERBOSE = False
EXTRA_PATH = ROOT / "gpurun_out" / "bench_extra.json"


def log(msg, always=False):
    """Progress on stderr: a few lines by default, every section with --verbose."""
    if always or VERBOSE:
        print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--quick", action="store_true", help="main step only (no extra sections, no CPU baseline)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--verbose", action="store_true", help="one progress line per section on stderr")
    p.add_argument("--only", default="",
                   help="comma-separated extra sections to run (default: all): fp64, physics, spaces, paper, "
                        "transposition, gather, plan, dedup, p2, p3, jacobian, assembly, fwdbwd, adjoint, batched")
    p.add_argument("--extra-out", default=str(EXTRA_PATH),
                   help="file that receives the full result with every extra section")
    return p.parse_args()


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update((ROOT / f).read_bytes())
    return h.hexdigest()[:16]


CSRC = "paper_1607_04245_amd/csrc/"
KERNEL_SOURCES = {
    "fem_integrate_residual_mesh": [CSRC + "residual_mesh.hip", CSRC + "mesh_kernel.hpp", CSRC + "fem_device.hpp",
                                    CSRC + "fem_scheme.hpp", CSRC + "fem_abi.hip"],
    "fem_integrate_residual": [CSRC + "residual_lane.hip", CSRC + "fem_device.hpp", CSRC + "fem_scheme.hpp",
                               CSRC + "fem_abi.hip"],
    "fem_geometry": [CSRC + "geometry.hip", CSRC + "fem_abi.hip"],
}


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    f = ROOT / "profiles" / "traffic.json"
    try:
        rec = json.loads(f.read_text())[f"{kernel}:{workload}"]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_hash") != source_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def main():
    global VERBOSE
    args = parse()
    VERBOSE = args.verbose
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}): the element stream shards with no "
              "communication, so each GPU would run this same single-GPU workload on its slice.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1607_04245_amd import _native as N, api, meshgen as mg, model

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    props = torch.cuda.get_device_properties(dev)
    log(f"device {props.name} {getattr(props, 'gcnArchName', '')} CUs {props.multi_processor_count} "
        f"mem {props.total_memory / 2**30:.0f} GiB", always=True)

    def to_dev(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def n_copies(bytes_per_copy):
        """Copies of a timed section's inputs, sized on the bytes its own
        kernel touches per launch: at least MIN_COPIES and more than
        ROTATE_BYTES in total, so that no launch finds its inputs in the
        256 MB last-level cache left behind by the launches before it."""
        if bytes_per_copy >= ROTATE_BYTES:
            return 2   # one launch alone overruns the last-level cache
        return int(max(MIN_COPIES, min(64, -(-ROTATE_BYTES // max(bytes_per_copy, 1)))))

    # -------------------------------------------------------------- main step --
    t0 = time.time()
    wl = mg.config(2)
    n, dim, phys, rule = wl.n_elem, wl.dim, wl.physics, wl.rule
    log(f"workload {wl.name}: {n} elements, {wl.n_vert} vertices (built in {time.time() - t0:.1f}s)")
    flops = model.model_flops(dim, phys, rule)

    def step_copies(dt):
        # sized on the fused kernel's bytes, the smallest per-launch footprint
        # of the kernels that rotate through these copies
        word = 4 if dt == torch.float32 else 8
        per = model.residual_mesh_bytes(dim, phys, rule, n, wl.n_vert, word) * n
        base = dict(coords=to_dev(wl.coords, torch.float64), conn=to_dev(wl.conn, torch.int32),
                    u=to_dev(wl.u, dt), coef=to_dev(wl.coef, dt))
        cs = []
        for _ in range(n_copies(per)):
            c = {k: v.clone() for k, v in base.items()}
            c["inv_j"] = torch.empty((dim * dim, n), dtype=dt, device=dev)
            c["det_j"] = torch.empty((n,), dtype=dt, device=dev)
            c["R"] = torch.empty_like(c["u"])
            cs.append(c)
        return cs

    def fused(c):
        api.fem_integrate_residual_mesh(dim, phys, rule, c["coords"], c["conn"], c["u"], c["coef"], out=c["R"])

    def geometry(c):
        api.fem_geometry(c["coords"], c["conn"], c["det_j"].dtype, inv_j=c["inv_j"], det_j=c["det_j"])

    def integrate(c):
        api.fem_integrate_residual(dim, phys, rule, c["inv_j"], c["det_j"], c["u"], c["coef"], out=c["R"])

    def graph_of(fn, cs, steps):
        """A HIP graph (torch's capture on the stream the library launches on)
        holding `steps` calls of fn rotating through the input copies."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for i in range(3):          # eager warm-up on the capture stream
                fn(cs[i % len(cs)])
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(steps):
                fn(cs[i % len(cs)])
        torch.cuda.synchronize()
        return g

    def timed_graph(fn, cs, steps, warmup):
        """The timed region: one replay of a graph of `steps` steps, bracketed
        by a pair of events; returns (wall seconds, event ms per step). Before
        it, the warm-up steps and then more replays until the GPU has run the
        section for PREHEAT_S: after the host work between sections the GPU
        has idled, and its first milliseconds of work run at lower clocks
        (the step measured 17.5-18.3 us per launch after 5 warm-up steps,
        15.9 us after 3000)."""
        g = graph_of(fn, cs, steps)
        for _ in range(max(1, warmup // steps + 1)):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < PREHEAT_S:
            g.replay()
            torch.cuda.synchronize()
        t = time.perf_counter()
        s = ev()
        g.replay()
        e = ev()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        return wall, s.elapsed_time(e) / steps

    def split(c):
        geometry(c)
        integrate(c)

    def breakdown(cs, reps=20):
        """Untimed: graphs of geometry alone and of integration alone."""
        _, g_ms = timed_graph(geometry, cs, reps, 1)
        _, i_ms = timed_graph(integrate, cs, reps, 1)
        return g_ms, i_ms

    cs = step_copies(torch.float32)
    wall, fused_ms = timed_graph(fused, cs, args.steps, args.warmup)
    swall, _ = timed_graph(split, cs, args.steps, args.warmup)
    geo_ms, int_ms = breakdown(cs)
    # for information: the same step on one copy, whose 74 MB then stay in
    # the 256 MB last-level cache between launches (the figures above rotate
    # through copies so that they do not)
    _, hot_ms = timed_graph(fused, cs[:1], args.steps, args.warmup)
    del cs
    ms_per_step = 1e3 * wall / args.steps
    value = n * args.steps / wall
    log(f"FP32 fused step {ms_per_step * 1e3:.1f} us ({value:.3e} elem/s), kernel {fused_ms * 1e3:.1f} us; "
        f"two-call step {1e6 * swall / args.steps:.1f} us (geometry {geo_ms * 1e3:.1f} us, integrate "
        f"{int_ms * 1e3:.1f} us); hot step (inputs cached) {hot_ms * 1e3:.1f} us", always=True)

    fused_bytes = model.residual_mesh_bytes(dim, phys, rule, n, wl.n_vert, 4) * n
    int_bytes = model.forward_bytes(dim, phys, rule, 4) * n
    geo_bytes = model.geometry_bytes(dim, n, wl.n_vert, 4) * n
    kernels = {
        "fem_integrate_residual_mesh": dict(avg_us=fused_ms * 1e3, algorithmic_bytes=fused_bytes,
                                            gbs=fused_bytes / (fused_ms * 1e-3) / 1e9,
                                            elements_per_s=n / (fused_ms * 1e-3),
                                            model_gflops=n * flops / (fused_ms * 1e-3) / 1e9),
        "fem_integrate_residual": dict(avg_us=int_ms * 1e3, algorithmic_bytes=int_bytes,
                                       gbs=int_bytes / (int_ms * 1e-3) / 1e9, elements_per_s=n / (int_ms * 1e-3),
                                       model_gflops=n * flops / (int_ms * 1e-3) / 1e9),
        "fem_geometry": dict(avg_us=geo_ms * 1e3, algorithmic_bytes=geo_bytes,
                             gbs=geo_bytes / (geo_ms * 1e-3) / 1e9, elements_per_s=n / (geo_ms * 1e-3)),
    }
    dom = "fem_integrate_residual_mesh"
    dk = kernels[dom]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic(dom, "laplace3d_2p20_f32"),
                "algorithmic_bytes_per_launch": dk["algorithmic_bytes"]}

    # ------------------------------------------------- achievable bandwidth --
    def copy_gbs(nbytes, reps):
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        k = 1 if nbytes >= 2**30 else n_copies(2 * nbytes)
        pairs = [(src if i == 0 else src.clone(), torch.empty_like(src)) for i in range(k)]
        _, ms = timed_graph(lambda p: api.fem_stream_copy(p[0], p[1]), pairs, reps, 1)
        return 2 * nbytes / (ms * 1e-3) / 1e9, ms * 1e3

    def rows_us(n_cols, n_in, n_out, dt, reps):
        """fem_stream_rows over the row structure of a kernel (n_in rows of
        n_cols words read, n_out written), rotated like the kernel's inputs."""
        word = 4 if dt == torch.float32 else 8
        k = n_copies((n_in + n_out) * n_cols * word)
        pairs = [(torch.ones(n_in, n_cols, dtype=dt, device=dev), torch.empty(n_out, n_cols, dtype=dt, device=dev))
                 for _ in range(k)]
        _, ms = timed_graph(lambda p: api.fem_stream_rows(p[0], p[1]), pairs, reps, 1)
        del pairs
        return ms * 1e3

    big_gbs, big_us = copy_gbs(2 << 30, 10)
    same_gbs, same_us = copy_gbs(int(dk["algorithmic_bytes"] // 2) // 16 * 16, 20)
    roofline["achievable_gbs"] = big_gbs
    roofline["frac_of_achievable"] = dk["gbs"] / big_gbs
    roofline["achievable_gbs_same_bytes"] = same_gbs
    log(f"copy: {big_gbs:.0f} GB/s on 2 GiB, {same_gbs:.0f} GB/s at the fused kernel's byte count", always=True)
    # the integrate-only kernel's rows (inverse Jacobian, det J, closure and
    # coefficient rows in; element-vector rows out) streamed without arithmetic
    nbt = api.n_basis(dim) * api.n_comp(dim, phys)
    int_rows = (dim * dim + 1 + nbt + api.n_coef(phys) * api.n_coef_words(dim, rule), nbt)
    kernels["fem_integrate_residual"]["stream_rows"] = list(int_rows)
    kernels["fem_integrate_residual"]["stream_rows_us"] = rows_us(n, int_rows[0], int_rows[1], torch.float32, 20)
    # the geometry kernel's bytes as rows: connectivity (dim + 1 words) and
    # the FP64 coordinates spread over the elements in; det J and J^{-1} out
    coord_words = max(1, round(8 * dim * wl.n_vert / (4 * n)))
    geo_rows = (dim + 1 + coord_words, dim * dim + 1)
    kernels["fem_geometry"]["stream_rows"] = list(geo_rows)
    kernels["fem_geometry"]["stream_rows_us"] = rows_us(n, geo_rows[0], geo_rows[1], torch.float32, 20)
    # and the fused kernel's: connectivity, coordinates, closure and
    # coefficient rows in, element-vector rows out
    mesh_rows = (dim + 1 + coord_words + nbt + api.n_coef(phys) * api.n_coef_words(dim, rule), nbt)
    roofline["same_rows_us"] = rows_us(n, mesh_rows[0], mesh_rows[1], torch.float32, 20)
    roofline["frac_of_rows"] = roofline["same_rows_us"] / dk["avg_us"]

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
                               "64^3 Kuhn grid, 4-point degree-2 rule; step = element residuals from coordinates, "
                               "connectivity, closure and coefficients (fem_integrate_residual_mesh: geometry and "
                               "integration in one pass)",
                   "n_elem": n, "n_vert": wl.n_vert},
        "model_gflops": value * flops / 1e9,
        "kernels": kernels,
        "roofline": roofline,
        "hot_step": dict(ms_per_step=hot_ms, elements_per_s=n / (hot_ms * 1e-3),
                         note="inputs left in the last-level cache between launches; information only"),
        "two_call_step": dict(elements_per_s=n * args.steps / swall, ms_per_step=1e3 * swall / args.steps,
                              note="fem_geometry (geometry stored) then fem_integrate_residual"),
        "stream_copy": dict(gbs_2gib=big_gbs, us_2gib=big_us, gbs_same_bytes=same_gbs, us_same_bytes=same_us),
    }

    only = {x.strip() for x in args.only.split(",") if x.strip()}

    def want(section):
        return not only or section in only

    if not args.quick:
        extra = {}

        # ------------------------------------------------------ FP64 step --
        if want("fp64"):
            cs = step_copies(torch.float64)
            steps64 = max(10, args.steps // 2)
            wall64, f64 = timed_graph(fused, cs, steps64, 2)
            swall64, _ = timed_graph(split, cs, steps64, 2)
            g64, i64 = breakdown(cs)
            del cs
            b64 = model.forward_bytes(dim, phys, rule, 8) * n
            fb64 = model.residual_mesh_bytes(dim, phys, rule, n, wl.n_vert, 8) * n
            extra["fp64_step"] = dict(elements_per_s=n * steps64 / wall64, ms_per_step=1e3 * wall64 / steps64,
                                      fused_us=f64 * 1e3, fused_gbs=fb64 / (f64 * 1e-3) / 1e9,
                                      fused_model_gflops=n * flops / (f64 * 1e-3) / 1e9,
                                      two_call_elements_per_s=n * steps64 / swall64,
                                      integrate_us=i64 * 1e3, integrate_gbs=b64 / (i64 * 1e-3) / 1e9,
                                      integrate_model_gflops=n * flops / (i64 * 1e-3) / 1e9, geometry_us=g64 * 1e3)
            # both kernels' rows streamed, in 8-byte words (the 16-byte
            # connectivity as two rows, the coordinates per element rounded)
            ncq = api.n_coef(phys) * api.n_coef_words(dim, rule)
            cw64 = max(1, round(8 * dim * wl.n_vert / (8 * n)))
            f64r = rows_us(n, (dim + 1) * 4 // 8 + cw64 + nbt + ncq, nbt, torch.float64, 20)
            i64r = rows_us(n, dim * dim + 1 + nbt + ncq, nbt, torch.float64, 20)
            extra["fp64_step"].update(fused_rows_us=f64r, fused_frac_of_rows=f64r / (f64 * 1e3),
                                      integrate_rows_us=i64r, integrate_frac_of_rows=i64r / (i64 * 1e3))
            log(f"FP64 fused step {extra['fp64_step']['ms_per_step'] * 1e3:.1f} us ({extra['fp64_step']['fused_gbs']:.0f}"
                f" GB/s; its rows streamed {f64r:.1f} us); integrate alone {i64 * 1e3:.1f} us "
                f"({extra['fp64_step']['integrate_gbs']:.0f} GB/s; rows {i64r:.1f} us)")

        # --------------------------------------------------- other physics --
        def integrate_only(wlx, dt, reps=20, space=mg.COEF_QUAD, coef=None):
            word = 4 if dt == torch.float32 else 8
            nb = model.forward_bytes(wlx.dim, wlx.physics, wlx.rule, word, coef_space=space) * wlx.n_elem
            ij, dj = api.fem_geometry(to_dev(wlx.coords, torch.float64), to_dev(wlx.conn, torch.int32), dt)
            base = dict(ij=ij, dj=dj, u=to_dev(wlx.u, dt), cf=to_dev(wlx.coef if coef is None else coef, dt))
            cps = []
            for _ in range(n_copies(nb)):
                c = {k: v.clone() for k, v in base.items()}
                c["R"] = torch.empty_like(c["u"])
                cps.append(c)
            del base, ij, dj

            def go(c):
                api.fem_integrate_residual(wlx.dim, wlx.physics, wlx.rule, c["ij"], c["dj"], c["u"], c["cf"],
                                           out=c["R"], coef_space=space)
            _, ms = timed_graph(go, cps, reps, 1)
            us = ms * 1e3
            r_in = sum(cps[0][key].numel() for key in ("ij", "dj", "u", "cf")) // wlx.n_elem
            r_out = cps[0]["u"].shape[0]
            del cps
            rw = rows_us(wlx.n_elem, r_in, r_out, dt, reps)
            f = model.model_flops(wlx.dim, wlx.physics, wlx.rule)
            return dict(n_elem=wlx.n_elem, us=us, gbs=nb / (us * 1e-6) / 1e9, elements_per_s=wlx.n_elem / (us * 1e-6),
                        model_gflops=wlx.n_elem * f / (us * 1e-6) / 1e9, frac_of_peak=nb / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                        stream_rows=[r_in, r_out], stream_rows_us=rw, frac_of_stream_rows=rw / us)

        def fused_only(wlx, dt, reps=20, space=mg.COEF_QUAD, coef=None):
            word = 4 if dt == torch.float32 else 8
            nb = model.residual_mesh_bytes(wlx.dim, wlx.physics, wlx.rule, wlx.n_elem, wlx.n_vert, word,
                                           coef_space=space) * wlx.n_elem
            base = dict(X=to_dev(wlx.coords, torch.float64), conn=to_dev(wlx.conn, torch.int32), u=to_dev(wlx.u, dt),
                        cf=to_dev(wlx.coef if coef is None else coef, dt))
            cps = []
            for _ in range(n_copies(nb)):
                c = {k: v.clone() for k, v in base.items()}
                c["R"] = torch.empty_like(c["u"])
                cps.append(c)
            del base

            def go(c):
                api.fem_integrate_residual_mesh(wlx.dim, wlx.physics, wlx.rule, c["X"], c["conn"], c["u"], c["cf"],
                                                out=c["R"], coef_space=space)
            _, ms = timed_graph(go, cps, reps, 1)
            us = ms * 1e3
            del cps
            f = model.model_flops(wlx.dim, wlx.physics, wlx.rule)
            return dict(n_elem=wlx.n_elem, us=us, gbs=nb / (us * 1e-6) / 1e9, elements_per_s=wlx.n_elem / (us * 1e-6),
                        model_gflops=wlx.n_elem * f / (us * 1e-6) / 1e9, frac_of_peak=nb / (us * 1e-6) / 1e9 / HBM_PEAK_GBS)

        if want("physics"):
            for cfg in ("3a", "3b"):
                wlx = mg.config(cfg)
                for dt, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
                    r = integrate_only(wlx, dt)
                    extra[f"{wlx.name}_{tag}_integrate"] = r
                    log(f"{wlx.name} {tag} integrate: {r['us']:.1f} us, {r['gbs']:.0f} GB/s, {r['model_gflops']:.0f} model GF/s")
                    r = fused_only(wlx, dt)
                    extra[f"{wlx.name}_{tag}_from_mesh"] = r
                    log(f"{wlx.name} {tag} from mesh: {r['us']:.1f} us ({r['elements_per_s']:.3e} elem/s), "
                        f"{r['gbs']:.0f} GB/s")
                del wlx

        # ---------------------------------------------- coefficient spaces --
        # The paper's GPU runs take the coefficient as a P1 field or per cell
        # (Section 4); P1 coefficients are the closure of a vertex field.
        if want("spaces"):
            for cfg in (2, "3a"):
                wlx = wl if cfg == 2 else mg.config(cfg)
                for space, sname in ((mg.COEF_P1, "p1"), (mg.COEF_P0, "p0")):
                    cf = mg.space_coefficients(wlx, space, mg.BASE_SEED + 1000)
                    r = integrate_only(wlx, torch.float32, space=space, coef=cf)
                    extra[f"{wlx.name}_f32_coef_{sname}_integrate"] = r
                    r2 = fused_only(wlx, torch.float32, space=space, coef=cf)
                    extra[f"{wlx.name}_f32_coef_{sname}_from_mesh"] = r2
                    log(f"{wlx.name} f32 coefficient {sname}: integrate {r['us']:.1f} us ({r['gbs']:.0f} GB/s), "
                        f"from mesh {r2['us']:.1f} us ({r2['elements_per_s']:.3e} elem/s, {r2['gbs']:.0f} GB/s)")
                    del cf
                del wlx

        # ----------------------------------------------------- paper analog --
        # The paper's headline case: 2D P1 Laplacian, variable coefficient in
        # the P1 space, one quadrature point (its flop model, Section 3), on
        # the 2^22-triangle mesh; model GF/s with the paper's per-cell formula.
        if want("paper"):
            wlp = mg.make_workload("laplace2d_2p22_centroid", 2, mg.LAPLACE, 1449, 1 << 22, mg.BASE_SEED + 6,
                                   rule=mg.RULE_CENTROID)
            cfp = mg.space_coefficients(wlp, mg.COEF_P1, mg.BASE_SEED + 1000)
            f1 = model.paper_flops_per_cell(2, 3, 1, 1)
            for dt, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
                r = integrate_only(wlp, dt, space=mg.COEF_P1, coef=cfp)
                r2 = fused_only(wlp, dt, space=mg.COEF_P1, coef=cfp)
                for rr in (r, r2):
                    rr["paper_model_gflops"] = rr["elements_per_s"] * f1 / 1e9
                extra[f"paper_analog_laplace2d_p1coef_nq1_{tag}_integrate"] = r
                extra[f"paper_analog_laplace2d_p1coef_nq1_{tag}_from_mesh"] = r2
                log(f"2D Laplacian, P1 coefficient, N_q = 1, {tag}: integrate {r['elements_per_s']:.3e} el/s "
                    f"({r['paper_model_gflops']:.0f} GF/s in the paper's model, {r['gbs']:.0f} GB/s), from mesh "
                    f"{r2['elements_per_s']:.3e} el/s ({r2['paper_model_gflops']:.0f} GF/s)")
            del wlp, cfp

        # ------------------------------------------ thread transposition --
        # The paper's strategy (Section 3: quadrature-point-parallel work, an
        # LDS transposition, basis-function-parallel work) against the default
        # one-element-per-lane kernel, on the step mesh and the paper's 2D
        # N_q = 1 case; best of the transposition's workgroup sizes.
        if want("transposition"):
            wlq = mg.make_workload("laplace2d_2p22_centroid", 2, mg.LAPLACE, 1449, 1 << 22, mg.BASE_SEED + 6,
                                   rule=mg.RULE_CENTROID)
            def best_of(wlx, strategy, shapes):
                """Fastest launch shape of a strategy: (shape, result) or None."""
                best = None
                for waves, bpc in shapes:
                    api.fem_set_tuning(wlx.dim, wlx.physics, wlx.rule, torch.float32, strategy=strategy, vec=1,
                                       waves_per_block=waves, blocks_per_cu=bpc)
                    try:
                        r = integrate_only(wlx, torch.float32)
                    except N.FemError:  # workgroup too large for this element's LDS tile
                        continue
                    if best is None or r["us"] < best[1]["us"]:
                        best = ((waves, bpc), r)
                return best

            shapes = [(w, b) for w in (1, 2, 4, 8) for b in (0, 2, 4, 8)]
            wle = mg.config("3b")   # 3D elasticity: the quad-permutation form covers scalar fields only
            for wlx, tag in ((wl, "laplace3d_2p20_f32"), (wlq, "laplace2d_2p22_centroid_f32"),
                             (wle, "elasticity3d_2p21_f32")):
                saved = api.fem_get_tuning(wlx.dim, wlx.physics, wlx.rule, torch.float32)
                lane = integrate_only(wlx, torch.float32)
                tt = best_of(wlx, N.STRATEGY_TRANSPOSE, shapes)
                sh = best_of(wlx, N.STRATEGY_SHUFFLE, shapes) if wlx.physics != mg.ELASTICITY else None
                api.fem_set_tuning(wlx.dim, wlx.physics, wlx.rule, torch.float32, **saved)
                rec = dict(lane_us=lane["us"], lane_gbs=lane["gbs"], transpose_us=tt[1]["us"],
                           transpose_gbs=tt[1]["gbs"], transpose_shape=tt[0])
                msg = (f"{tag}: lane kernel {lane['us']:.1f} us ({lane['gbs']:.0f} GB/s), thread transposition "
                       f"through LDS {tt[1]['us']:.1f} us ({tt[1]['gbs']:.0f} GB/s, shape {tt[0]})")
                if sh is not None:
                    rec.update(shuffle_us=sh[1]["us"], shuffle_gbs=sh[1]["gbs"], shuffle_shape=sh[0])
                    msg += f", through quad permutations {sh[1]['us']:.1f} us ({sh[1]['gbs']:.0f} GB/s, shape {sh[0]})"
                extra[f"strategies_{tag}"] = rec
                log(msg, always=True)
            del wlq, wle

        # ------------------------------------------------------ gather form --
        # u per vertex (and a P1 coefficient per vertex), gathered in the kernel.
        def gather_only(wlx, dt, space, reps=20):
            word = 4 if dt == torch.float32 else 8
            nb = model.residual_gather_bytes(wlx.dim, wlx.physics, wlx.rule, wlx.n_elem, wlx.n_vert, word,
                                             coef_space=space) * wlx.n_elem
            s = mg.BASE_SEED + 1000
            cg = mg.vertex_coefficients(wlx, s) if space == mg.COEF_P1 else mg.space_coefficients(wlx, space, s)
            base = dict(X=to_dev(wlx.coords, torch.float64), conn=to_dev(wlx.conn, torch.int32),
                        u=to_dev(wlx.u_vertex, dt), cf=to_dev(cg, dt))
            nbt = wlx.u.shape[0]
            cps = []
            for _ in range(n_copies(nb)):
                c = {k: v.clone() for k, v in base.items()}
                c["R"] = torch.empty((nbt, wlx.n_elem), dtype=dt, device=dev)
                cps.append(c)
            del base

            def go(c):
                api.fem_integrate_residual_gather(wlx.dim, wlx.physics, wlx.rule, c["X"], c["conn"], c["u"], c["cf"],
                                                  out=c["R"], coef_space=space)
            _, ms = timed_graph(go, cps, reps, 1)
            us = ms * 1e3
            del cps
            f = model.model_flops(wlx.dim, wlx.physics, wlx.rule)
            return dict(n_elem=wlx.n_elem, us=us, gbs=nb / (us * 1e-6) / 1e9, elements_per_s=wlx.n_elem / (us * 1e-6),
                        model_gflops=wlx.n_elem * f / (us * 1e-6) / 1e9, bytes_per_elem=nb / wlx.n_elem,
                        frac_of_peak=nb / (us * 1e-6) / 1e9 / HBM_PEAK_GBS)

        if want("gather"):
            for cfg in (2, "3b"):
                wlx = wl if cfg == 2 else mg.config(cfg)
                for space, sname in ((mg.COEF_QUAD, "quad"), (mg.COEF_P1, "p1")):
                    for dt, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
                        r = gather_only(wlx, dt, space)
                        extra[f"{wlx.name}_{tag}_coef_{sname}_gather"] = r
                        log(f"{wlx.name} {tag} gather, coefficient {sname}: {r['us']:.1f} us "
                            f"({r['elements_per_s']:.3e} elem/s, {r['bytes_per_elem']:.1f} B/elem, {r['gbs']:.0f} GB/s)")
                del wlx

        # ------------------------------------------------------- mesh plans --
        # The from-mesh residual through a per-mesh plan of each tile's
        # distinct vertices (built once, outside the timed region; its build
        # time is reported), beside the unplanned fused and gather kernels.
        if want("plan"):
            for cfg in (2, "3a", "3b"):
                wlx = wl if cfg == 2 else mg.config(cfg)
                conn0 = to_dev(wlx.conn, torch.int32)
                t0 = time.perf_counter()
                plan0 = api.MeshPlan(conn0, wlx.n_vert)
                build_s = time.perf_counter() - t0
                info = plan0.info()
                plan0.close()
                for dt, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
                    word = 4 if dt == torch.float32 else 8
                    row = dict(n_elem=wlx.n_elem, plan_build_s=build_s, tile_vertices_per_elem=info["tile_vertices"] / wlx.n_elem)
                    for gather in (False, True):
                        nb = model.planned_bytes(wlx.dim, wlx.physics, wlx.rule, wlx.n_elem, wlx.n_vert,
                                                 info["tile_vertices"], word, gather=gather) * wlx.n_elem
                        base = dict(X=to_dev(wlx.coords, torch.float64), conn=conn0,
                                    u=to_dev(wlx.u_vertex if gather else wlx.u, dt), cf=to_dev(wlx.coef, dt))
                        cps = []
                        for _ in range(n_copies(nb)):
                            c = {k: v.clone() for k, v in base.items()}
                            c["plan"] = api.MeshPlan(c["conn"], wlx.n_vert)
                            c["R"] = torch.empty(wlx.u.shape, dtype=dt, device=dev)
                            cps.append(c)
                        del base

                        def go(c, wlx=wlx, gather=gather):
                            f = c["plan"].gather if gather else c["plan"].integrate
                            f(wlx.physics, wlx.rule, c["X"], c["u"], c["cf"], out=c["R"])
                        _, ms = timed_graph(go, cps, 20, 1)
                        for c in cps:
                            c["plan"].close()
                        del cps
                        unplanned = (gather_only(wlx, dt, mg.COEF_QUAD) if gather else fused_only(wlx, dt))["us"]
                        form = "gather" if gather else "closure"
                        row[f"{form}_us"] = ms * 1e3
                        row[f"{form}_elements_per_s"] = wlx.n_elem / (ms * 1e-3)
                        row[f"{form}_gbs"] = nb / (ms * 1e-3) / 1e9
                        row[f"{form}_unplanned_us"] = unplanned
                    # the geometry alone, through the plan and through fem_geometry
                    nb = model.geometry_bytes(wlx.dim, wlx.n_elem, wlx.n_vert, word) * wlx.n_elem
                    cps = []
                    for _ in range(n_copies(nb)):
                        c = dict(X=to_dev(wlx.coords, torch.float64), conn=conn0.clone())
                        c["plan"] = api.MeshPlan(c["conn"], wlx.n_vert)
                        c["ij"] = torch.empty((wlx.dim * wlx.dim, wlx.n_elem), dtype=dt, device=dev)
                        c["dj"] = torch.empty((wlx.n_elem,), dtype=dt, device=dev)
                        cps.append(c)

                    def geo_plain(c, dt=dt):
                        api.fem_geometry(c["X"], c["conn"], dt, inv_j=c["ij"], det_j=c["dj"])

                    def geo_planned(c, dt=dt):
                        c["plan"].geometry(c["X"], dt, inv_j=c["ij"], det_j=c["dj"])
                    _, ms_g = timed_graph(geo_plain, cps, 20, 1)
                    _, ms_gp = timed_graph(geo_planned, cps, 20, 1)
                    for c in cps:
                        c["plan"].close()
                    del cps
                    row.update(geometry_us=ms_gp * 1e3, geometry_unplanned_us=ms_g * 1e3,
                               geometry_gbs=nb / (ms_gp * 1e-3) / 1e9)
                    extra[f"{wlx.name}_{tag}_mesh_plan"] = row
                    log(f"{wlx.name} {tag} mesh plan (built in {build_s:.2f} s, "
                        f"{row['tile_vertices_per_elem']:.2f} tile vertices per element): closure "
                        f"{row['closure_us']:.1f} us (unplanned {row['closure_unplanned_us']:.1f}), gather "
                        f"{row['gather_us']:.1f} us (unplanned {row['gather_unplanned_us']:.1f}), geometry "
                        f"{row['geometry_us']:.1f} us (unplanned {row['geometry_unplanned_us']:.1f})")
                del conn0, wlx

        # ------------------------------------------- run-time vertex dedup --
        # The fused from-mesh residual with each wave's distinct vertices
        # gathered once into LDS (FEM_STRATEGY_DEDUP), against the per-lane
        # gathers of the default strategy; best of a few launch shapes.
        if want("dedup"):
            for cfg in (2, "3a", "3b"):
                wlx = wl if cfg == 2 else mg.config(cfg)
                for dt, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
                    saved = api.fem_get_tuning(wlx.dim, wlx.physics, wlx.rule, dt, op=N.OP_RESIDUAL_MESH)
                    lane = fused_only(wlx, dt)
                    best = None
                    for waves, bpc in ((2, 0), (4, 0), (2, 8), (4, 4)):
                        api.fem_set_tuning(wlx.dim, wlx.physics, wlx.rule, dt, strategy=N.STRATEGY_DEDUP, vec=1,
                                           waves_per_block=waves, blocks_per_cu=bpc, op=N.OP_RESIDUAL_MESH)
                        r = fused_only(wlx, dt)
                        if best is None or r["us"] < best[1]["us"]:
                            best = ((waves, bpc), r)
                    api.fem_set_tuning(wlx.dim, wlx.physics, wlx.rule, dt, op=N.OP_RESIDUAL_MESH, **saved)
                    extra[f"{wlx.name}_{tag}_dedup"] = dict(lane_us=lane["us"], lane_gbs=lane["gbs"],
                                                             dedup_us=best[1]["us"], dedup_gbs=best[1]["gbs"],
                                                             dedup_shape=best[0])
                    log(f"{wlx.name} {tag} from mesh: per-lane gathers {lane['us']:.1f} us ({lane['gbs']:.0f} GB/s), "
                        f"run-time dedup {best[1]['us']:.1f} us ({best[1]['gbs']:.0f} GB/s, shape {best[0]})",
                        always=True)
                del wlx

        # ------------------------------------------------- second order (P2) --
        if want("p2"):
            for cfg, rule_p2 in ((2, mg.RULE_TET11), ("3b", mg.RULE_TET11), ("3a", mg.RULE_TRI6)):
                wlx = wl if cfg == 2 else mg.config(cfg)
                p2 = mg.p2_inputs(wlx, rule_p2, mg.BASE_SEED + 5000)
                for dt, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
                    word = 4 if dt == torch.float32 else 8
                    nb = model.p2_forward_bytes(wlx.dim, wlx.physics, rule_p2, word) * wlx.n_elem
                    ij, dj = api.fem_geometry(to_dev(wlx.coords, torch.float64), to_dev(wlx.conn, torch.int32), dt)
                    base = dict(ij=ij, dj=dj, u=to_dev(p2.u, dt), cf=to_dev(p2.coef, dt))
                    cps = []
                    for _ in range(n_copies(nb)):
                        c = {k: v.clone() for k, v in base.items()}
                        c["R"] = torch.empty_like(c["u"])
                        cps.append(c)
                    del base

                    def go(c, wlx=wlx, rule_p2=rule_p2):
                        api.fem_integrate_residual_p2(wlx.dim, wlx.physics, rule_p2, c["ij"], c["dj"], c["u"], c["cf"],
                                                      out=c["R"])
                    _, ms = timed_graph(go, cps, 20, 1)
                    us = ms * 1e3
                    f = model.p2_model_flops(wlx.dim, wlx.physics, rule_p2)
                    # a copy of the same bytes: how much of the kernel's time the
                    # stream itself needs, whatever unit does the arithmetic
                    cp_gbs, cp_us = copy_gbs(int(nb // 2) // 16 * 16, 20)
                    # and the same rows streamed without arithmetic
                    r_in = sum(cps[0][key].numel() for key in ("ij", "dj", "u", "cf")) // wlx.n_elem
                    r_out = cps[0]["u"].shape[0]
                    rw_us = rows_us(wlx.n_elem, r_in, r_out, dt, 20)
                    extra[f"{wlx.name}_p2_{tag}_integrate"] = dict(
                        n_elem=wlx.n_elem, rule=rule_p2, us=us, gbs=nb / (us * 1e-6) / 1e9,
                        elements_per_s=wlx.n_elem / (us * 1e-6), model_gflops=wlx.n_elem * f / (us * 1e-6) / 1e9,
                        bytes_per_elem=nb / wlx.n_elem, copy_same_bytes_us=cp_us, frac_of_copy_same_bytes=cp_us / us,
                        stream_rows=[r_in, r_out], stream_rows_us=rw_us, frac_of_stream_rows=rw_us / us)
                    log(f"{wlx.name} P2 {tag} integrate: {us:.1f} us ({wlx.n_elem / (us * 1e-6):.3e} elem/s, "
                        f"{nb / (us * 1e-6) / 1e9:.0f} GB/s, {wlx.n_elem * f / (us * 1e-6) / 1e12:.1f} model TF/s); "
                        f"copy of the same bytes {cp_us:.1f} us, the same {r_in} + {r_out} rows streamed {rw_us:.1f} us")
                    del cps, ij, dj
                del p2, wlx

        # -------------------------------------------------- third order (P3) --
        if want("p3"):
            for cfg in (2, "3b", "3a"):
                wlx = wl if cfg == 2 else mg.config(cfg)
                rule_p3 = mg.RULE_TET11 if wlx.dim == 3 else mg.RULE_TRI6
                p3 = mg.p3_inputs(wlx, rule_p3, mg.BASE_SEED + 7700)
                for dt, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
                    word = 4 if dt == torch.float32 else 8
                    nb = model.p3_forward_bytes(wlx.dim, wlx.physics, rule_p3, word) * wlx.n_elem
                    ij, dj = api.fem_geometry(to_dev(wlx.coords, torch.float64), to_dev(wlx.conn, torch.int32), dt)
                    base = dict(ij=ij, dj=dj, u=to_dev(p3.u, dt), cf=to_dev(p3.coef, dt))
                    cps = []
                    for _ in range(n_copies(nb)):
                        c = {k: v.clone() for k, v in base.items()}
                        c["R"] = torch.empty_like(c["u"])
                        cps.append(c)
                    del base

                    def go(c, wlx=wlx, rule_p3=rule_p3):
                        api.fem_integrate_residual_p3(wlx.dim, wlx.physics, rule_p3, c["ij"], c["dj"], c["u"], c["cf"],
                                                      out=c["R"])
                    saved = api.fem_get_tuning(wlx.dim, wlx.physics, rule_p3, dt, op=N.OP_RESIDUAL_P3)
                    api.fem_set_tuning(wlx.dim, wlx.physics, rule_p3, dt, op=N.OP_RESIDUAL_P3, strategy=N.STRATEGY_LANE,
                                       vec=1, waves_per_block=1 if wlx.dim == 3 else 4, blocks_per_cu=0)
                    _, ms = timed_graph(go, cps, 10, 1)
                    us = ms * 1e3
                    mfma = None
                    if wlx.dim == 3:
                        # the transposition on the matrix cores, best launch shape
                        for waves, bpc in ((1, 0), (2, 0), (4, 0), (4, 2), (4, 4), (2, 4)):
                            api.fem_set_tuning(wlx.dim, wlx.physics, rule_p3, dt, op=N.OP_RESIDUAL_P3,
                                               strategy=N.STRATEGY_MFMA, vec=1, waves_per_block=waves, blocks_per_cu=bpc)
                            _, msm = timed_graph(go, cps, 10, 1)
                            if mfma is None or msm * 1e3 < mfma[1]:
                                mfma = ((waves, bpc), msm * 1e3)
                    comp = None
                    if wlx.dim == 3 and wlx.physics == mg.ELASTICITY:
                        # three waves per tile, one per component, best launch shape
                        shapes = ((1, 0), (1, 2), (1, 4), (1, 8)) + (((2, 0), (2, 2), (2, 4)) if tag == "f32" else ())
                        for waves, bpc in shapes:
                            api.fem_set_tuning(wlx.dim, wlx.physics, rule_p3, dt, op=N.OP_RESIDUAL_P3,
                                               strategy=N.STRATEGY_COMPONENT, vec=1, waves_per_block=waves,
                                               blocks_per_cu=bpc)
                            _, msc = timed_graph(go, cps, 10, 1)
                            if comp is None or msc * 1e3 < comp[1]:
                                comp = ((waves, bpc), msc * 1e3)
                    api.fem_set_tuning(wlx.dim, wlx.physics, rule_p3, dt, op=N.OP_RESIDUAL_P3, **saved)
                    f = model.p3_model_flops(wlx.dim, wlx.physics, rule_p3)
                    cp_gbs, cp_us = copy_gbs(int(nb // 2) // 16 * 16, 10)
                    # the same rows streamed without arithmetic: geometry, closure
                    # and coefficient rows in, the element-vector rows out
                    nbt = c["u"].shape[0]
                    r_in = sum(c[key].numel() for key in ("ij", "dj", "u", "cf")) // wlx.n_elem
                    rw_us = rows_us(wlx.n_elem, r_in, nbt, dt, 10)
                    extra[f"{wlx.name}_p3_{tag}_integrate"] = dict(
                        n_elem=wlx.n_elem, rule=rule_p3, us=us, gbs=nb / (us * 1e-6) / 1e9,
                        elements_per_s=wlx.n_elem / (us * 1e-6), model_gflops=wlx.n_elem * f / (us * 1e-6) / 1e9,
                        bytes_per_elem=nb / wlx.n_elem, copy_same_bytes_us=cp_us, frac_of_copy_same_bytes=cp_us / us,
                        stream_rows=[r_in, nbt], stream_rows_us=rw_us, frac_of_stream_rows=rw_us / us)
                    if mfma:
                        extra[f"{wlx.name}_p3_{tag}_integrate"].update(
                            mfma_us=mfma[1], mfma_shape=mfma[0], mfma_gbs=nb / (mfma[1] * 1e-6) / 1e9,
                            mfma_frac_of_copy_same_bytes=cp_us / mfma[1])
                    if comp:
                        extra[f"{wlx.name}_p3_{tag}_integrate"].update(
                            component_us=comp[1], component_shape=comp[0], component_gbs=nb / (comp[1] * 1e-6) / 1e9,
                            component_frac_of_copy_same_bytes=cp_us / comp[1])
                    log(f"{wlx.name} P3 {tag} integrate: lane kernel {us:.1f} us ({wlx.n_elem / (us * 1e-6):.3e} elem/s, "
                        f"{nb / (us * 1e-6) / 1e9:.0f} GB/s, {wlx.n_elem * f / (us * 1e-6) / 1e12:.1f} model TF/s)"
                        + (f", matrix-core transposition {mfma[1]:.1f} us (shape {mfma[0]})" if mfma else "")
                        + (f", component lanes {comp[1]:.1f} us (shape {comp[0]})" if comp else "")
                        + f"; copy of the same bytes {cp_us:.1f} us, the same {r_in} + {nbt} rows streamed "
                          f"{rw_us:.1f} us", always=wlx.dim == 3)
                    if wlx.dim == 3:
                        # the adjoint (du and dcoef) on the same inputs, w a
                        # separate copy of u (its own rows, as a caller's would be)
                        nbb = model.p3_backward_bytes(wlx.dim, wlx.physics, rule_p3, word) * wlx.n_elem
                        for c in cps:
                            c["dc"] = torch.empty_like(c["cf"])
                            c["w"] = c["u"].clone()

                        def back(c, wlx=wlx, rule_p3=rule_p3):
                            api.fem_integrate_residual_p3_backward(wlx.dim, wlx.physics, rule_p3, c["ij"], c["dj"], c["u"],
                                                                   c["cf"], c["w"], du=c["R"], dcoef=c["dc"])
                        _, msb = timed_graph(back, cps, 10, 1)
                        ncq = c["cf"].numel() // wlx.n_elem
                        rb_us = rows_us(wlx.n_elem, r_in + nbt, nbt + ncq, dt, 10)
                        extra[f"{wlx.name}_p3_{tag}_adjoint"] = dict(
                            n_elem=wlx.n_elem, us=msb * 1e3, gbs=nbb / (msb * 1e-3) / 1e9, bytes_per_elem=nbb / wlx.n_elem,
                            stream_rows_us=rb_us, frac_of_stream_rows=rb_us / (msb * 1e3))
                        log(f"{wlx.name} P3 {tag} adjoint: {msb * 1e3:.1f} us ({nbb / (msb * 1e-3) / 1e9:.0f} GB/s); "
                            f"its rows streamed {rb_us:.1f} us")
                    del cps, ij, dj
                del p3, wlx

        # ------------------------------------------------- element matrices --
        if want("jacobian"):
            for cfg, order, rule_k, dts in ((2, 1, mg.RULE_TET4, ("f32", "f64")), (2, 2, mg.RULE_TET11, ("f32", "f64")),
                                          ("3b", 1, mg.RULE_TET4, ("f32", "f64")), ("3b", 2, mg.RULE_TET11, ("f32",)),
                                          (2, 3, mg.RULE_TET11, ("f32",))):
                wlx = wl if cfg == 2 else mg.config(cfg)
                cf0 = mg.p2_inputs(wlx, rule_k, mg.BASE_SEED + 5000).coef
                nbt = model.n_basis(wlx.dim, order) * wlx.n_comp
                for tag in dts:
                    dt = torch.float32 if tag == "f32" else torch.float64
                    word = 4 if dt == torch.float32 else 8
                    nb = model.jacobian_bytes(wlx.dim, wlx.physics, rule_k, word, order=order) * wlx.n_elem
                    ij, dj = api.fem_geometry(to_dev(wlx.coords, torch.float64), to_dev(wlx.conn, torch.int32), dt)
                    base = dict(ij=ij, dj=dj, cf=to_dev(cf0, dt))
                    cps = []
                    for _ in range(n_copies(nb)):
                        c = {k: v.clone() for k, v in base.items()}
                        c["K"] = torch.empty((nbt * nbt, wlx.n_elem), dtype=dt, device=dev)
                        cps.append(c)
                    del base, ij, dj

                    def go(c, wlx=wlx, rule_k=rule_k, order=order):
                        api.fem_integrate_jacobian(wlx.dim, wlx.physics, rule_k, c["ij"], c["dj"], c["cf"], out=c["K"],
                                                   order=order)
                    _, ms = timed_graph(go, cps, 10, 1)
                    us = ms * 1e3
                    rec = extra[f"{wlx.name}_jacobian_p{order}_{tag}"] = dict(
                        n_elem=wlx.n_elem, rule=rule_k, us=us, gbs=nb / (us * 1e-6) / 1e9,
                        elements_per_s=wlx.n_elem / (us * 1e-6), bytes_per_elem=nb / wlx.n_elem,
                        frac_of_peak=nb / (us * 1e-6) / 1e9 / HBM_PEAK_GBS)
                    del cps
                    # the same rows streamed (geometry and coefficient rows in,
                    # one row per matrix entry out), where the yardstick takes them
                    n_in = wlx.dim * wlx.dim + 1 + cf0.size // wlx.n_elem
                    if nbt * nbt <= 256:
                        rec["stream_rows_us"] = rows_us(wlx.n_elem, n_in, nbt * nbt, dt, 10)
                        rec["frac_of_stream_rows"] = rec["stream_rows_us"] / us
                    log(f"{wlx.name} element matrices P{order} {tag}: {us:.1f} us ({wlx.n_elem / (us * 1e-6):.3e} elem/s, "
                        f"{nb / wlx.n_elem:.0f} B/elem, {nb / (us * 1e-6) / 1e9:.0f} GB/s)")
                del cf0, wlx

        # --------------------------------------------------------- assembly --
        # global residual: element vectors summed onto vertices (deterministic gather)
        if want("assembly"):
            for cfg in (2, "3b"):
                wlx = wl if cfg == 2 else mg.config(cfg)
                nc = wlx.n_comp
                conn_d = to_dev(wlx.conn, torch.int32)
                plan = api.AssemblyPlan(conn_d, wlx.n_vert)
                nb = model.assemble_bytes(wlx.dim, nc, wlx.n_elem, wlx.n_vert, 4) * wlx.n_elem
                R0 = torch.randn(((wlx.dim + 1) * nc, wlx.n_elem), device=dev)
                cps = [dict(R=R0.clone(), F=torch.empty((wlx.n_vert, nc), device=dev)) for _ in range(n_copies(nb))]
                del R0

                def go(c, plan=plan, nc=nc):
                    plan.assemble(c["R"], nc, out=c["F"])
                _, ms = timed_graph(go, cps, 20, 1)
                us = ms * 1e3
                extra[f"{wlx.name}_f32_assemble"] = dict(n_elem=wlx.n_elem, n_vert=wlx.n_vert, us=us,
                                                         gbs=nb / (us * 1e-6) / 1e9,
                                                         elements_per_s=wlx.n_elem / (us * 1e-6))
                log(f"{wlx.name} f32 assembly: {us:.1f} us ({nb / (us * 1e-6) / 1e9:.0f} GB/s)")
                del cps, plan, conn_d, wlx

        # ------------------------------------- forward and adjoint, one step --
        # Every row of the path on the step workload: the fused residual
        # (storing the geometry), then the adjoint (du and dcoef) of
        # L = sum w . R from that geometry.
        if want("fwdbwd"):
            dt = torch.float32
            nb_fb = (model.residual_mesh_bytes(dim, phys, rule, n, wl.n_vert, 4, store_geometry=True)
                     + model.backward_bytes(dim, phys, rule, 4)) * n
            base = dict(X=to_dev(wl.coords, torch.float64), conn=to_dev(wl.conn, torch.int32), u=to_dev(wl.u, dt),
                        cf=to_dev(wl.coef, dt), w=to_dev(wl.w, dt))
            cps = []
            for _ in range(n_copies(nb_fb)):
                c = {k: v.clone() for k, v in base.items()}
                c["R"], c["du"], c["dc"] = torch.empty_like(c["u"]), torch.empty_like(c["u"]), torch.empty_like(c["cf"])
                c["ij"], c["dj"] = torch.empty((dim * dim, n), dtype=dt, device=dev), torch.empty(n, dtype=dt, device=dev)
                cps.append(c)
            del base

            def fwd_bwd(c):
                api.fem_integrate_residual_mesh(dim, phys, rule, c["X"], c["conn"], c["u"], c["cf"], out=c["R"],
                                                inv_j=c["ij"], det_j=c["dj"])
                api.fem_integrate_residual_backward(dim, phys, rule, c["ij"], c["dj"], c["u"], c["cf"], c["w"],
                                                    du=c["du"], dcoef=c["dc"])
            _, ms = timed_graph(fwd_bwd, cps, 20, 1)
            for c in cps:
                c["plan"] = api.MeshPlan(c["conn"], wl.n_vert)

            def fwd_bwd_planned(c):
                c["plan"].integrate(phys, rule, c["X"], c["u"], c["cf"], out=c["R"], inv_j=c["ij"], det_j=c["dj"])
                api.fem_integrate_residual_backward(dim, phys, rule, c["ij"], c["dj"], c["u"], c["cf"], c["w"],
                                                    du=c["du"], dcoef=c["dc"])
            _, ms_p = timed_graph(fwd_bwd_planned, cps, 20, 1)
            for c in cps:
                c["plan"].close()
            extra["forward_and_adjoint_step_laplace3d_2p20_f32"] = dict(
                us=ms * 1e3, elements_per_s=n / (ms * 1e-3), algorithmic_bytes=nb_fb, gbs=nb_fb / (ms * 1e-3) / 1e9,
                with_mesh_plan_us=ms_p * 1e3)
            log(f"forward (geometry stored) and adjoint, one step: {ms * 1e3:.1f} us ({n / (ms * 1e-3):.3e} elem/s, "
                f"{nb_fb / (ms * 1e-3) / 1e9:.0f} GB/s); with a mesh plan {ms_p * 1e3:.1f} us")
            del cps

        # --------------------------------------------------------- adjoint --
        if want("adjoint"):
            wl5 = mg.config(5)
            dt = torch.float32
            nb = model.backward_bytes(3, mg.LAPLACE, wl5.rule, 4) * wl5.n_elem
            ij, dj = api.fem_geometry(to_dev(wl5.coords, torch.float64), to_dev(wl5.conn, torch.int32), dt)
            base = dict(ij=ij, dj=dj, u=to_dev(wl5.u, dt), cf=to_dev(wl5.coef, dt), w=to_dev(wl5.w, dt))
            cps = []
            for _ in range(n_copies(nb)):
                c = {k: v.clone() for k, v in base.items()}
                c["du"], c["dc"] = torch.empty_like(c["u"]), torch.empty_like(c["cf"])
                cps.append(c)
            del base, ij, dj

            def bwd(c):
                api.fem_integrate_residual_backward(3, mg.LAPLACE, wl5.rule, c["ij"], c["dj"], c["u"], c["cf"], c["w"],
                                                    du=c["du"], dcoef=c["dc"])
            _, ms = timed_graph(bwd, cps, 20, 1)
            us = ms * 1e3
            rec = extra["adjoint_laplace3d_2p21_f32"] = dict(n_elem=wl5.n_elem, us=us, gbs=nb / (us * 1e-6) / 1e9,
                                                             elements_per_s=wl5.n_elem / (us * 1e-6),
                                                             frac_of_peak=nb / (us * 1e-6) / 1e9 / HBM_PEAK_GBS)
            del cps
            # its rows streamed: geometry, u, coefficient and w rows in; du and
            # dcoef rows out
            nbt5 = api.n_basis(3) * api.n_comp(3, mg.LAPLACE)
            ncq5 = api.n_coef(mg.LAPLACE) * api.n_coef_words(3, wl5.rule)
            rec["stream_rows_us"] = rows_us(wl5.n_elem, 10 + 2 * nbt5 + ncq5, nbt5 + ncq5, dt, 20)
            rec["frac_of_stream_rows"] = rec["stream_rows_us"] / us
            log(f"adjoint: {us:.1f} us, {nb / (us * 1e-6) / 1e9:.0f} GB/s; its rows streamed {rec['stream_rows_us']:.1f} us")
            del wl5

        # --------------------------------------------------------- batched --
        if want("batched"):
            t0 = time.time()
            wls = mg.batch_workloads()
            dt = torch.float32
            meshes, nbytes, ntot = [], 0, 0
            for w in wls:
                ij, dj = api.fem_geometry(to_dev(w.coords, torch.float64), to_dev(w.conn, torch.int32), dt)
                meshes.append(dict(dim=w.dim, physics=w.physics, rule=w.rule, inv_j=ij, det_j=dj, u=to_dev(w.u, dt),
                                   coef=to_dev(w.coef, dt), out=torch.empty(w.u.shape, dtype=dt, device=dev)))
                nbytes += model.forward_bytes(w.dim, w.physics, w.rule, 4) * w.n_elem
                ntot += w.n_elem
            del wls
            log(f"batched: {len(meshes)} meshes, {ntot} elements, {nbytes / 1e6:.0f} MB (built in {time.time() - t0:.1f}s)")

            def separate():
                for m in meshes:
                    api.fem_integrate_residual(m["dim"], m["physics"], m["rule"], m["inv_j"], m["det_j"], m["u"],
                                               m["coef"], out=m["out"])

            plan = api.BatchPlan(meshes)
            side = torch.cuda.Stream()
            with torch.cuda.stream(side):
                shape = plan.autotune()   # launch shape from the plan's own meshes
                plan.capture()
            torch.cuda.synchronize()

            def timeit(fn, reps, stream=None):
                for _ in range(3):
                    fn()
                torch.cuda.synchronize()
                pairs = []
                for _ in range(reps):
                    s = ev()
                    fn()
                    pairs.append((s, ev()))
                torch.cuda.synchronize()
                return 1e3 * sorted(a.elapsed_time(b) for a, b in pairs)[reps // 2]

            def replay():
                plan.replay()

            sep_us = timeit(separate, 10)
            _, sep_graph_ms = timed_graph(lambda _: separate(), [0], 5, 1)
            run_us = timeit(plan.run, 10)
            with torch.cuda.stream(side):
                rep_us = timeit(replay, 10)
            plan.close()
            extra["batched_64_meshes_f32"] = dict(
                n_mesh=len(meshes), n_elem=ntot, algorithmic_bytes=nbytes,
                separate_launches_us=sep_us, separate_launches_in_a_graph_us=sep_graph_ms * 1e3,
                persistent_launch_us=run_us, graph_replay_us=rep_us,
                graph_replay_gbs=nbytes / (rep_us * 1e-6) / 1e9, graph_replay_elements_per_s=ntot / (rep_us * 1e-6),
                speedup_vs_separate=sep_graph_ms * 1e3 / rep_us,
                speedup_vs_separate_issued_from_python=sep_us / rep_us, autotuned_launch=shape,
                note="speedup_vs_separate: the 64 single-mesh launches recorded in one graph against the one "
                     "persistent launch; the meshes total about 0.9 GB, above the last-level cache; medians of 10")
            log(f"batched: 64 launches {sep_us:.1f} us ({sep_graph_ms * 1e3:.1f} us as one graph), persistent "
                f"{run_us:.1f} us, graph {rep_us:.1f} us "
                f"({nbytes / (rep_us * 1e-6) / 1e9:.0f} GB/s, {sep_graph_ms * 1e3 / rep_us:.2f}x the graph of 64); "
                f"autotuned launch {shape}", always=True)
            del meshes
        result["extra"] = extra

    if not args.quick and not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(wl, flops)

    # The full record, every extra section included, goes to a file; stdout
    # gets one compact line, last.
    out = pathlib.Path(args.extra_out)
    try:
        out.parent.mkdir(parents=True, exist_ok=True)
        out.write_text(json.dumps(result, indent=1))
        result["extra_file"] = str(out.relative_to(ROOT) if out.is_relative_to(ROOT) else out)
    except OSError as exc:
        log(f"could not write {out}: {exc}", always=True)
    print(json.dumps(compact(result)), flush=True)


def _r(x, digits=4):
    """x rounded to `digits` significant digits (None stays None)."""
    return None if x is None else float(f"{x:.{digits}g}")


def compact(res):
    """The stdout record: the contract's keys, the roofline of the step's
    kernel, the CPU baseline, and one short object per headline variant
    (FP64 step, integrate-only kernel, two-call step, copy yardstick,
    batched launch, thread transposition, elasticity)."""
    rf = res["roofline"]
    k = res["kernels"]
    line = {key: res[key] for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                                      "higher_is_better", "scaling", "vs_baseline", "dtype", "data")}
    line["value"] = _r(line["value"], 6)
    line["ms_per_step"] = _r(line["ms_per_step"], 5)
    line["config"] = {"workload": res["config"]["workload"], "n_elem": res["config"]["n_elem"],
                      "n_vert": res["config"]["n_vert"]}
    line["model_gflops"] = _r(res["model_gflops"])
    line["roofline"] = {"bound": rf["bound"], "kernel": rf["kernel"], "achieved": _r(rf["achieved"]),
                        "peak": rf["peak"], "unit": rf["unit"], "frac": _r(rf["frac"]),
                        "traffic": rf["traffic"], "algorithmic_bytes_per_launch": rf["algorithmic_bytes_per_launch"],
                        "kernel_us": _r(k[rf["kernel"]]["avg_us"]), "achievable_gbs": _r(rf.get("achievable_gbs")),
                        "frac_of_achievable": _r(rf.get("frac_of_achievable")),
                        "copy_same_bytes_gbs": _r(rf.get("achievable_gbs_same_bytes"))}
    if "same_rows_us" in rf:
        line["roofline"]["same_rows_us"] = _r(rf["same_rows_us"])
        line["roofline"]["frac_of_rows"] = _r(rf["frac_of_rows"])
    ki = k["fem_integrate_residual"]
    line["integrate_only"] = {"kernel": "fem_integrate_residual", "us": _r(ki["avg_us"]),
                              "elements_per_s": _r(ki["elements_per_s"]), "gbs": _r(ki["gbs"]),
                              "frac": _r(ki["gbs"] / HBM_PEAK_GBS), "model_gflops": _r(ki["model_gflops"]),
                              "algorithmic_bytes_per_launch": ki["algorithmic_bytes"]}
    if "stream_rows_us" in ki:
        line["integrate_only"]["rows_us"] = _r(ki["stream_rows_us"])
        line["integrate_only"]["frac_of_rows"] = _r(ki["stream_rows_us"] / ki["avg_us"])
    kg = k["fem_geometry"]
    line["geometry_only"] = {"us": _r(kg["avg_us"]), "gbs": _r(kg["gbs"]), "frac": _r(kg["gbs"] / HBM_PEAK_GBS)}
    if "stream_rows_us" in kg:
        line["geometry_only"]["rows_us"] = _r(kg["stream_rows_us"])
        line["geometry_only"]["frac_of_rows"] = _r(kg["stream_rows_us"] / kg["avg_us"])
    line["two_call_step"] = {"elements_per_s": _r(res["two_call_step"]["elements_per_s"]),
                             "ms_per_step": _r(res["two_call_step"]["ms_per_step"])}
    if "hot_step" in res:
        line["hot_step"] = {"elements_per_s": _r(res["hot_step"]["elements_per_s"]),
                            "ms_per_step": _r(res["hot_step"]["ms_per_step"])}
    ex = res.get("extra", {})
    if "fp64_step" in ex:
        f = ex["fp64_step"]
        line["fp64"] = {"value": _r(f["elements_per_s"]), "ms_per_step": _r(f["ms_per_step"]),
                        "kernel_us": _r(f["fused_us"]), "frac": _r(f["fused_gbs"] / HBM_PEAK_GBS),
                        "integrate_us": _r(f["integrate_us"]), "integrate_frac": _r(f["integrate_gbs"] / HBM_PEAK_GBS)}
        if "fused_frac_of_rows" in f:
            line["fp64"]["frac_of_rows"] = _r(f["fused_frac_of_rows"])
            line["fp64"]["integrate_frac_of_rows"] = _r(f["integrate_frac_of_rows"])
    el = {}
    for key, tag in (("elasticity2d_2p22_f32_integrate", "2d_f32"), ("elasticity3d_2p21_f32_integrate", "3d_f32"),
                     ("elasticity2d_2p22_f64_integrate", "2d_f64"), ("elasticity3d_2p21_f64_integrate", "3d_f64")):
        if key in ex:
            el[tag] = {"elements_per_s": _r(ex[key]["elements_per_s"]), "frac": _r(ex[key]["frac_of_peak"])}
            if "frac_of_stream_rows" in ex[key]:
                el[tag]["frac_of_rows"] = _r(ex[key]["frac_of_stream_rows"])
    if el:
        line["elasticity_integrate"] = el
    if "adjoint_laplace3d_2p21_f32" in ex:
        a = ex["adjoint_laplace3d_2p21_f32"]
        line["adjoint"] = {"us": _r(a["us"]), "frac": _r(a["frac_of_peak"])}
        if "frac_of_stream_rows" in a:
            line["adjoint"]["frac_of_rows"] = _r(a["frac_of_stream_rows"])
    if "batched_64_meshes_f32" in ex:
        b = ex["batched_64_meshes_f32"]
        line["batched"] = {"graph_replay_us": _r(b["graph_replay_us"]),
                           "elements_per_s": _r(b["graph_replay_elements_per_s"]),
                           "frac": _r(b["graph_replay_gbs"] / HBM_PEAK_GBS),
                           "separate_in_one_graph_us": _r(b["separate_launches_in_a_graph_us"]),
                           "speedup_vs_separate": _r(b["speedup_vs_separate"])}
    tt = {k2[len("strategies_"):]: {"lane_us": _r(v["lane_us"]), "lds_us": _r(v["transpose_us"]),
                                     **({"shuffle_us": _r(v["shuffle_us"])} if "shuffle_us" in v else {})}
          for k2, v in ex.items() if k2.startswith("strategies_")}
    p3 = {}
    for key, v in ex.items():
        if key.endswith("_integrate") and "_p3_" in key and "mfma_us" in v:
            p3[key[:-len("_integrate")]] = {"lane_us": _r(v["us"]), "mfma_us": _r(v["mfma_us"]),
                                            "copy_us": _r(v["copy_same_bytes_us"])}
            if "component_us" in v:
                p3[key[:-len("_integrate")]]["component_us"] = _r(v["component_us"])
            if "stream_rows_us" in v:
                p3[key[:-len("_integrate")]]["rows_us"] = _r(v["stream_rows_us"])
    if p3:
        line["p3_transposition"] = p3
    if tt:
        line["transposition"] = tt
    cb = res.get("cpu_baseline")
    if cb:
        line["cpu_baseline"] = {"value": _r(cb["value"]), "unit": cb["unit"], "cores": cb["cores"], "kind": cb["kind"],
                                "sample": cb["sample"],
                                "single_thread": _r(cb["single_thread"]["value"])}
    if "extra_file" in res:
        line["extra_file"] = res["extra_file"]
    # stay below MAX_LINE bytes whatever the variants hold: drop the optional
    # objects last-added first
    for key in ("p3_transposition", "transposition", "elasticity_integrate", "adjoint", "geometry_only",
                "two_call_step", "hot_step", "batched"):
        if len(json.dumps(line)) <= MAX_LINE:
            break
        line.pop(key, None)
    return line


def cpu_baseline(wl, flops):
    """The FP64 oracle (plain C, unchanged) on the step's work: geometry and
    residual of every element of the step workload. All host cores: the
    elements are split into one contiguous chunk per thread and each thread
    calls the oracle on its chunk (the C routine runs outside Python's
    interpreter lock); one warm-up pass, then the median of five passes.
    One thread: the same call over all elements, repeated for about 8 s."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    bounds = np.linspace(0, wl.n_elem, threads + 1).astype(np.int64)
    chunks = [(np.ascontiguousarray(wl.conn[a:b]), np.ascontiguousarray(wl.u[:, a:b]),
               np.ascontiguousarray(wl.coef[:, :, a:b])) for a, b in zip(bounds[:-1], bounds[1:])]

    def one(ch):
        R, nd = oracle.residual(wl.dim, wl.physics, wl.rule, wl.coords, ch[0], ch[1], ch[2])
        return nd, bool(np.isfinite(R).all())

    times = []
    with cf.ThreadPoolExecutor(threads) as ex:
        for rep in range(6):
            t = time.perf_counter()
            res = list(ex.map(one, chunks))
            if rep:
                times.append(time.perf_counter() - t)
    assert all(nd == 0 and ok for nd, ok in res)
    eps_mt = wl.n_elem / float(np.median(times))

    reps, t_total = 0, 0.0
    while t_total < 8.0 and reps < 50:
        t = time.perf_counter()
        R, nd = oracle.residual(wl.dim, wl.physics, wl.rule, wl.coords, wl.conn, wl.u, wl.coef)
        t_total += time.perf_counter() - t
        reps += 1
    assert nd == 0 and np.isfinite(R).all()
    eps_1 = wl.n_elem * reps / t_total
    log(f"CPU oracle: {eps_mt:.3e} elements/s on {threads} threads, {eps_1:.3e} on one", always=True)
    return {"value": eps_mt, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": f"fem_oracle_residual (FP64 geometry + residual) over all {wl.n_elem} elements of the step "
                      f"workload, split into {threads} contiguous chunks on {threads} threads; median of 5 passes "
                      f"after one warm-up",
            "model_gflops": eps_mt * flops / 1e9,
            "single_thread": {"value": eps_1, "passes": reps, "seconds": t_total,
                              "model_gflops": eps_1 * flops / 1e9},
            "host_cpus_visible": os.cpu_count()}


if __name__ == "__main__":
    main()
