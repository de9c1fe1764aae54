#!/usr/bin/env python
"""Benchmark: GLL points/s through Q-criterion + isosurface extraction.

One step = the whole extraction path over one synthetic snapshot already
resident in HBM: one sem_extract call (Q, |omega|, per-element Q range, and
the cull / classify / scan-compact / emit of the triangles of every
isovalue, fused in a single pass).  The same work as two calls
(sem_qcrit, then sem_isosurface) is timed beside it for comparison.  Workload: the turbulent-channel snapshot -- 64 x 32 x 32 = 65,536
order-7 hexahedra (33,554,432 GLL points), tanh wall stretching (beta = 2),
parabolic mean plus a seeded random-phase k^-5/3 velocity field -- with Q
isosurfaces at the 90th, 95th and 99th percentiles of Q.

Prints ONE JSON line.  `roofline` describes the dominant kernel (its
average duration measured with HIP events on the launch stream);
`cpu_baseline` times the CPU FP64 oracle on a bounded sample of the same
snapshot.  One GPU only: --gpus above 1 exits with a message.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "extract_channel65536_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2312_09888_amd", "csrc", "sem_kernels.hip")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", choices=("f64", "f32"), default="f64")
    ap.add_argument("--cpu-baseline", choices=("on", "off"), default="on")
    ap.add_argument("--cpu-elements", type=int, default=16384,
                    help="elements of the snapshot the CPU oracle is timed on")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (a kernel of "
                         "known HBM traffic for scaling profiler byte counters)")
    return ap.parse_args()


def log(args, *msg):
    if not args.quiet:
        print(*msg, file=sys.stderr, flush=True)


def kernel_sha():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(n_launch_points):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, or None
    when the kernel source changed after the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_src_sha256") != kernel_sha():
        return None
    if rec.get("points_per_launch") != n_launch_points:
        return None
    return rec.get("hbm_bytes_per_launch")


def load_isovalues():
    with open(os.path.join(ROOT, "tests", "golden", "channel_isovalues.json")) as fh:
        rec = json.load(fh)
    return rec["isovalues"], rec["percentiles"]


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the element-parallel extraction needs no communication; see the "
              "sharding design).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2312_09888_amd as sem
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    devn = "cuda:0"
    torch.cuda.set_device(0)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    n = 7
    shape = W.CHANNEL_SHAPE
    n_elem = shape[0] * shape[1] * shape[2]
    p3 = (n + 1) ** 3
    points = n_elem * p3
    isos, pcts = load_isovalues()

    t0 = time.time()
    fields = W.channel_config(n, shape=shape, device=devn)
    fields = [f.to(tdt).contiguous() for f in fields]
    x, y, z, u, v, w = fields
    torch.cuda.synchronize()
    log(args, f"inputs generated on GPU in {time.time() - t0:.1f} s "
              f"({points} points, {args.dtype})")

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=devn).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(args, "copy calibration: 1 GiB read + 1 GiB written")
        del src, dst

    sem.init(0)
    k_iso = len(isos)
    dcode = sem.SEM_F64 if args.dtype == "f64" else sem.SEM_F32
    q = torch.empty_like(u)
    om = torch.empty_like(u)
    mm = torch.empty((n_elem, 2), dtype=tdt, device=devn)
    status = torch.zeros(1, dtype=torch.int32, device=devn)
    ws = torch.empty(sem.extract_workspace_bytes(n_elem, n, k_iso, dcode), dtype=torch.uint8,
                     device=devn)
    cnt = torch.zeros(k_iso, dtype=torch.int64, device=devn)
    act = torch.zeros(k_iso, dtype=torch.int64, device=devn)

    # exact triangle counts once (untimed count-only call), then buffers
    sem.extract_into(x, y, z, u, v, w, isos, [None] * k_iso, cnt, ws, active=act)
    torch.cuda.synchronize()
    counts = cnt.cpu().tolist()
    total_tri = int(sum(counts))
    tris = [torch.empty((c, 3, 3), dtype=tdt, device=devn) for c in counts]
    log(args, f"isovalues {isos} -> triangles {counts}, active cells {act.cpu().tolist()}")

    def step():
        sem.extract_into(x, y, z, u, v, w, isos, tris, cnt, ws, q=q, omega_mag=om,
                         minmax=mm, status=status)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(args, f"warmup {args.warmup} steps done")

    evs = []
    torch.cuda.synchronize()
    t_begin = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_begin.record()
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        evs.append((e0, e1))
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_begin.elapsed_time(t_end)
    ms_step = total_ms / args.steps
    k_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    flags = int(status.item())
    if flags:
        print(f"device status flags set: {flags}", file=sys.stderr)
        sys.exit(1)
    if cnt.cpu().tolist() != counts:
        print("triangle counts changed between steps", file=sys.stderr)
        sys.exit(1)
    log(args, f"timed {args.steps} steps: {ms_step:.4f} ms/step "
              f"(sem_extract launch average {k_ms:.4f} ms)")

    # the same path as two calls (sem_qcrit, then sem_isosurface), for comparison
    iws = torch.empty(sem.workspace_bytes(n_elem, n, k_iso), dtype=torch.uint8, device=devn)
    tri_all = torch.empty((max(total_tri, 1), 3, 3), dtype=tdt, device=devn)
    reps = max(3, args.steps // 4)
    torch.cuda.synchronize()
    a0 = torch.cuda.Event(enable_timing=True)
    a1 = torch.cuda.Event(enable_timing=True)
    a2 = torch.cuda.Event(enable_timing=True)
    qc_ms = iso_ms = 0.0
    for _ in range(reps):
        a0.record()
        sem.qcrit(x, y, z, u, v, w, q=q, omega_mag=om, minmax=mm)
        a1.record()
        sem.isosurface_into(x, y, z, q, isos, tri_all, cnt, iws, minmax=mm)
        a2.record()
        torch.cuda.synchronize()
        qc_ms += a0.elapsed_time(a1) / reps
        iso_ms += a1.elapsed_time(a2) / reps
    log(args, f"two-call path: sem_qcrit {qc_ms:.4f} ms + sem_isosurface {iso_ms:.4f} ms")

    esz = 8 if args.dtype == "f64" else 4
    # algorithmic bytes of one fused launch: read x,y,z,u,v,w, write Q,
    # |omega|, the per-element (min, max) and 9 coordinates per triangle
    k_bytes = points * 8 * esz + n_elem * 2 * esz + total_tri * 9 * esz
    k_gbs = k_bytes / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic(points)
    roof = {
        "bound": "hbm",
        "kernel": f"extract_pencil<7,{'double' if esz == 8 else 'float'}>",
        "achieved": round(k_gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(k_gbs / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "avg_ms": round(k_ms, 5),
        "algorithmic_bytes_per_launch": k_bytes,
    }
    result = {
        "metric": "GLL points/sec through Q-criterion+isosurface, % HBM roofline, plain vs mixed",
        "value": points / (ms_step * 1e-3),
        "unit": "GLL points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": "turbulent channel 64x32x32 hex elements, order 7, "
                        "33,554,432 GLL points, Q isosurfaces at 3 percentiles",
            "n_elem": n_elem, "order": n, "points": points,
            "isovalues": isos, "percentiles": pcts, "triangles": counts,
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "two_call_ms": {"sem_qcrit": round(qc_ms, 5), "sem_isosurface": round(iso_ms, 5)},
    }

    if args.cpu_baseline == "on":
        result["cpu_baseline"] = cpu_baseline(args, fields, isos, n, n_elem)
    print(json.dumps(result), flush=True)


def cpu_baseline(args, fields, isos, n, n_elem):
    """Time the CPU FP64 oracle (qcrit + isosurface) on a sample of elements."""
    import numpy as np

    from oracle import gll, mc
    from oracle import sem as osem

    k = min(args.cpu_elements, n_elem)
    rng = np.random.default_rng(0)
    els = np.sort(rng.choice(n_elem, size=k, replace=False))
    idx = __import__("torch").from_numpy(els).to(fields[0].device)
    arrs = [f.index_select(0, idx).double().cpu().numpy() for f in fields]
    d = gll.diff_matrix(n)
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    t0 = time.perf_counter()
    q, om, _ = osem.qcrit(*arrs, d)
    mc.extract(*arrs[:3], q, isos)
    dt_s = time.perf_counter() - t0
    pts = k * (n + 1) ** 3
    log(args, f"cpu oracle: {k} elements in {dt_s:.2f} s with {threads} threads")
    return {"value": pts / dt_s, "unit": "GLL points/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{k} random elements of the same snapshot ({pts} points), "
                      f"FP64 numpy oracle, Q + |omega| + {len(isos)} isosurfaces, "
                      f"{dt_s:.2f} s"}


if __name__ == "__main__":
    main()
