#!/usr/bin/env python
"""Benchmark: GLL points/s through Q-criterion + isosurface extraction.

One step = the whole extraction path over one synthetic snapshot already
resident in HBM: one sem_extract call (Q, |omega|, per-element Q range, and
the cull / classify / scan-compact / emit of the triangles of every
isovalue, fused in a single pass).  The K timed steps run as HIP graphs
(the steps' kernels captured once, up to 100 steps per graph, each graph
replayed once); the same steps launched eagerly, and the same work as two
calls (sem_qcrit, then sem_isosurface), are timed beside them for
comparison.  Workload: the turbulent-channel snapshot -- 64 x 32 x 32 = 65,536
order-7 hexahedra (33,554,432 GLL points), tanh wall stretching (beta = 2),
parabolic mean plus a seeded random-phase k^-5/3 velocity field -- with Q
isosurfaces at the 90th, 95th and 99th percentiles of Q.

Prints ONE JSON line.  `roofline` describes the dominant kernel (its
average duration measured with HIP events that the library records on the
launch stream around each kernel phase, over the timed steps);
`cpu_baseline` times the CPU FP64 oracle on a bounded sample of the same
snapshot.  One GPU only: --gpus above 1 exits with a message.

Two helper modes turn rocprofv3 CSV output into the committed summaries:
  --summarize-trace DIR OUT   kernel-trace statistics (run_kernel_stats.csv)
  --summarize-pmc FETCH_DIR WRITE_DIR OUT
                              FETCH_SIZE / WRITE_SIZE runs of
                              `bench.py --copy-calibration`, scaled by what the
                              counters read for the 1 GiB calibration copy.
  --summarize-mfma DIR OUT    matrix-core counters (SQ_INSTS_VALU_MFMA_MOPS_*)
                              of the mixed-precision Q kernels per mode.
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
KERNEL_SRC = os.path.join(ROOT, "paper_2312_09888_amd", "csrc", "sem_kernels.hip")
CALIBRATION_BYTES = 1 << 30


def traffic_file(kernel, dtype):
    # named for the kernel without its template arguments
    base = kernel.split("<")[0]
    return os.path.join(ROOT, "profiles", f"{base}_channel65536_{dtype}_traffic.json")


# kernel that runs the Q phase of sem_extract for order 7
def q_kernel_name(dtype):
    return "qcount_dma7<true>" if dtype == "f64" else "qcrit_pencil<7, float>"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dtype", choices=("f64", "f32"), default="f64")
    ap.add_argument("--cpu-baseline", choices=("on", "off"), default="on")
    ap.add_argument("--precision-modes", choices=("on", "off"), default="on",
                    help="also time FP32 and the mixed-precision modes on the same snapshot")
    ap.add_argument("--c0", choices=("on", "off"), default="on",
                    help="also time C0 averaging of Q and welding of the isosurfaces")
    ap.add_argument("--batched", choices=("on", "off"), default="on",
                    help="also time 16 uneven snapshots (orders 5/7/9) in one persistent "
                         "launch, and the whole batched step replayed as a HIP graph")
    ap.add_argument("--compression", choices=("on", "off"), default="on",
                    help="also train the per-element autoencoder and time compression of "
                         "a 262,144-element FP32 snapshot against the modal baseline")
    ap.add_argument("--cpu-elements", type=int, default=65536,
                    help="elements of the snapshot the CPU oracle is timed on")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (a kernel of "
                         "known HBM traffic for scaling profiler byte counters)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("DIR", "OUT"))
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"))
    ap.add_argument("--summarize-mfma", nargs=2, metavar=("DIR", "OUT"))
    ap.add_argument("--command", default="",
                    help="command line recorded in a summary (with --summarize-*)")
    return ap.parse_args()


def log(args, *msg):
    if not args.quiet:
        print(*msg, file=sys.stderr, flush=True)


def kernel_sha():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(kernel, dtype, n_launch_points):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, or None
    when the kernel source changed after the counters were taken."""
    try:
        with open(traffic_file(kernel, dtype)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_src_sha256") != kernel_sha():
        return None
    if rec.get("points_per_launch") != n_launch_points:
        return None
    return rec.get("hbm_bytes_per_launch")


MFMA_FILE = os.path.join(ROOT, "profiles", "mixed7_channel65536_mfma.json")
MIX_MODES = {"0": "bf16", "1": "fp16", "2": "bf16x3", "3": "fp16x3"}
MFMA_PEAK_TFLOPS = 2500.0     # MI355X dense BF16 / FP16 matrix peak


def measured_mfma():
    """Matrix-core FLOPs per launch of each mixed mode's Q kernel from the
    committed counter summary, or {} when the kernel source changed."""
    try:
        with open(MFMA_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return {}
    if rec.get("kernel_src_sha256") != kernel_sha():
        return {}
    return {m: v["mfma_flops_per_launch"] for m, v in rec.get("modes", {}).items()}


def load_isovalues():
    with open(os.path.join(ROOT, "tests", "golden", "channel_isovalues.json")) as fh:
        rec = json.load(fh)
    return rec["isovalues"], rec["percentiles"]


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, args.command)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.command)
        return
    if args.summarize_mfma:
        summarize_mfma(*args.summarize_mfma, args.command)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the element-parallel extraction needs no communication between "
              "GPUs; each would take its own share of the elements).  Run with "
              "--gpus 1.", file=sys.stderr)
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
    # every launch goes to a stream of its own: on the legacy default stream
    # the host now and then blocked inside launches for most of a step,
    # leaving the GPU idle between kernels (1.37 against 0.97 ms per step)
    bench_stream = torch.cuda.Stream()
    torch.cuda.set_stream(bench_stream)
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

    sem.init(0)
    if args.copy_calibration:
        src = torch.empty(CALIBRATION_BYTES // 8, dtype=torch.float64, device=devn).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        sem.stream_copy(src, dst)
        torch.cuda.synchronize()
        log(args, "copy calibration: 1 GiB read + 1 GiB written by stream_copy16")
        del src, dst
    copy_bw = copy_bandwidth(args, sem, devn)

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

    t_begin = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)

    # kernel-phase timing over K steps: the library launches each phase's
    # kernels with HIP events stamped from their dispatch timestamps, on the
    # launch stream.  The stamping leaves short gaps between kernels, so
    # these steps give the per-kernel durations, not the headline figure.
    torch.cuda.synchronize()
    sem.timing_begin(4 * args.steps + 16)
    t_begin.record()
    for _ in range(args.steps):
        step()
    t_end.record()
    torch.cuda.synchronize()
    phases, dropped = sem.timing_end()
    ms_phased = t_begin.elapsed_time(t_end) / args.steps
    if dropped:
        print(f"phase timing dropped {dropped} spans", file=sys.stderr)
        sys.exit(1)
    phase_ms = {k: (ms / c if c else 0.0) for k, (ms, c) in phases.items()}
    log(args, f"with phase timing: {ms_phased:.4f} ms/step; per-phase averages "
              + ", ".join(f"{k} {v:.4f} ms" for k, v in phase_ms.items() if v))

    # the timed steps (the headline figure), without phase events
    torch.cuda.synchronize()
    t_begin.record()
    h0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    t_end.record()
    host_ms = (time.perf_counter() - h0) * 1e3 / args.steps
    torch.cuda.synchronize()
    ms_step = t_begin.elapsed_time(t_end) / args.steps
    flags = int(status.item())
    if flags:
        print(f"device status flags set: {flags}", file=sys.stderr)
        sys.exit(1)
    if cnt.cpu().tolist() != counts:
        print("triangle counts changed between steps", file=sys.stderr)
        sys.exit(1)
    log(args, f"eager {args.steps} steps: {ms_step:.4f} ms/step (host enqueue {host_ms:.4f} "
              "ms/step)")

    # the timed steps (the headline figure): the K steps' kernels captured
    # in HIP graphs of up to 100 steps each and replayed once.  Eager steps
    # leave the GPU idle whenever the host is slow to launch (now and then
    # about 1 ms per step on the same box, against 0.04 ms); one replay per
    # step still adds a gap per replay.
    def capture(m):
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                for _ in range(m):
                    step()
        torch.cuda.current_stream().wait_stream(side)
        return g

    per_graph = min(args.steps, 100)
    graphs = [capture(per_graph)] * (args.steps // per_graph)
    if args.steps % per_graph:
        graphs.append(capture(args.steps % per_graph))
    for g in set(graphs):
        g.replay()
    torch.cuda.synchronize()
    t_begin.record()
    for g in graphs:
        g.replay()
    t_end.record()
    torch.cuda.synchronize()
    ms_graph = t_begin.elapsed_time(t_end) / args.steps
    if int(status.item()) or cnt.cpu().tolist() != counts:
        print("graph replays changed the status or the triangle counts", file=sys.stderr)
        sys.exit(1)
    log(args, f"timed {args.steps} steps in graph replays: {ms_graph:.4f} ms/step")
    del graphs

    # per-step timing protocol: single steps bracketed by their own events,
    # warm (back to back) and cold (L2 and MALL flushed before each step by
    # a 512 MiB copy that touches 1 GiB); median and the 10th / 90th
    # percentiles over the repetitions
    protocol = step_protocol(args, sem, step, devn)
    log(args, "per-step protocol: " + ", ".join(
        f"{k} median {v['median_ms']:.4f} ms (p10 {v['p10_ms']:.4f}, p90 {v['p90_ms']:.4f})"
        for k, v in protocol.items() if isinstance(v, dict)))

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
    # dominant kernel: the Q phase of sem_extract.  Algorithmic bytes of one
    # launch: read x, y, z, u, v, w; write Q and |omega| at every point, the
    # (min, max) of Q per element and (fused for order 7 FP64) one int32
    # triangle count per (isovalue, element).
    kname = q_kernel_name(args.dtype)
    k_ms = phase_ms["qcrit"]
    k_bytes = points * 8 * esz + n_elem * 2 * esz + (k_iso * n_elem * 4 if esz == 8 else 0)
    k_gbs = k_bytes / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic(kname, args.dtype, points)
    # the whole step: 64 (FP64) / 32 (FP32) B per point and 72 / 36 B per
    # triangle
    step_bytes = points * 8 * esz + total_tri * 9 * esz
    step_gbs = step_bytes / (ms_graph * 1e-3) / 1e9
    roof = {
        "bound": "hbm",
        "kernel": kname,
        "achieved": round(k_gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(k_gbs / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "copy_gbps": round(copy_bw, 1),
        "frac_of_copy": round(k_gbs / copy_bw, 4),
        "avg_ms": round(k_ms, 5),
        "algorithmic_bytes_per_launch": k_bytes,
        "dominant": max(phase_ms, key=phase_ms.get) == "qcrit",
    }
    result = {
        "metric": "GLL points/sec through Q-criterion+isosurface, % HBM roofline, plain vs mixed",
        "value": points / (ms_graph * 1e-3),
        "unit": "GLL points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_graph, 5),
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
        "phase_ms": {k: round(v, 5) for k, v in phase_ms.items() if v},
        "launch": "HIP graphs of up to 100 steps (the steps' kernels captured once), "
                  "each replayed once",
        "step_hbm": {"algorithmic_bytes": step_bytes,
                     "achieved_gbps": round(step_gbs, 1),
                     "frac_of_peak": round(step_gbs / HBM_PEAK_GBS, 4),
                     "frac_of_copy": round(step_gbs / copy_bw, 4)},
        "copy_bandwidth_gbps": round(copy_bw, 1),
        "step_protocol": protocol,
        "eager_ms_per_step": round(ms_step, 5),
        "ms_per_step_with_phase_timing": round(ms_phased, 5),
        "two_call_ms": {"sem_qcrit": round(qc_ms, 5), "sem_isosurface": round(iso_ms, 5)},
        "build": build_record(sem),
    }

    if args.batched == "on" and args.dtype == "f64":
        result["batched"] = batched_timing(args, sem)
    if args.c0 == "on" and args.dtype == "f64":
        result["c0"] = c0_timing(args, sem, fields, q, isos, n)
    if args.precision_modes == "on" and args.dtype == "f64":
        result["precision_modes"] = precision_modes(args, sem, fields, isos, n_elem, points)
    if args.compression == "on" and args.dtype == "f64":
        result["compression"] = compression_timing(args, sem)
    if args.cpu_baseline == "on":
        result["cpu_baseline"] = cpu_baseline(args, fields, isos, n, n_elem)
    print(json.dumps(result), flush=True)


def _pcts(ms):
    import numpy as np
    a = np.asarray(ms, dtype=np.float64)
    return {"median_ms": round(float(np.median(a)), 5),
            "p10_ms": round(float(np.percentile(a, 10)), 5),
            "p90_ms": round(float(np.percentile(a, 90)), 5)}


def build_record(sem):
    """The loaded library's build record (sem_build_info) and whether its
    sources digest is that of the sources in this tree."""
    from paper_2312_09888_amd import build as B
    rec = sem.build_info()
    rec["library"] = os.path.relpath(sem.lib()._name, ROOT)
    rec["matches_tree_sources"] = rec.get("sources_sha256") == B.source_sha256()
    return rec


def copy_bandwidth(args, sem, dev, nbytes=CALIBRATION_BYTES, reps=20):
    """Sustained HBM bandwidth of the library's plain copy kernel
    (sem_stream_copy): nbytes read and nbytes written per call, median over
    `reps` calls each bracketed by events."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ms = []
    for r in range(reps + 2):
        e0.record()
        sem.stream_copy(src, dst)
        e1.record()
        torch.cuda.synchronize()
        if r >= 2:
            ms.append(e0.elapsed_time(e1))
    med = _pcts(ms)["median_ms"]
    gbps = 2 * nbytes / (med * 1e-3) / 1e9
    log(args, f"stream copy: {2 * nbytes / 2**30:.1f} GiB moved in {med:.4f} ms (median of "
              f"{reps}): {gbps:.1f} GB/s = {gbps / HBM_PEAK_GBS:.3f} of the HBM peak")
    del src, dst
    return gbps


def step_protocol(args, sem, step, dev, reps=60):
    """Single steps, each between its own pair of events: warm (back to
    back) and cold (a 512 MiB copy before each step evicts L2 and the
    256 MB MALL)."""
    import torch
    flush_a = torch.empty(1 << 27, dtype=torch.float32, device=dev).fill_(0.0)
    flush_b = torch.empty_like(flush_a)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    out = {"reps": reps, "warmup": 5}
    for mode in ("warm", "cold"):
        for _ in range(5):
            step()
        torch.cuda.synchronize()
        for a, b in ev:
            if mode == "cold":
                sem.stream_copy(flush_a, flush_b)
            a.record()
            step()
            b.record()
        torch.cuda.synchronize()
        out[mode] = _pcts([a.elapsed_time(b) for a, b in ev])
    del flush_a, flush_b
    return out


def compression_timing(args, sem):
    """Learned in-transit compression of a 262,144-element order-7 FP32
    snapshot (u, v, w of the Taylor-Green vortex and a Gaussian random
    scalar theta, advected; 134 M points).  Training on the GPU: a pool of
    16,384 elements drawn from the 64 training phases, layer-wise PCA
    initialisation, then Adam on the max-error loss; the PCA-initialised
    network's fallback is reported beside the trained one's.  The snapshot is a held-out time (phase
    63.5): compressed and decompressed, against the Legendre modal baseline
    with the same bytes per element; agreement of the Q isosurface (90th
    percentile) of the decompressed velocity with the original's."""
    import numpy as np
    import torch

    import workloads as W
    dev = "cuda:0"
    t0 = time.time()
    ph, el = W.ae_training_elements(0, 16384)
    pools = []
    for p in np.unique(ph):
        f = W.ae_fields(int(p), dev, elements=el[ph == p], dtype=torch.float32)
        pools.append(sem.ae_blocks(list(f))[0])
    pool = torch.cat(pools)
    del pools
    torch.cuda.synchronize()
    t_pool = time.time() - t0

    def clock(fn):
        torch.cuda.synchronize()
        a = time.time()
        out = fn()
        torch.cuda.synchronize()
        return out, time.time() - a

    (params, _), t_pca = clock(lambda: sem.ae_pca_init(pool))
    params_pca = params.clone()
    eval_idx = torch.arange(4096, device=dev)
    max_loss = sem.SEM_AE_LOSS_MAX

    def losses(p):
        return (float(sem.ae_grad(pool, p, idx=eval_idx)[0].item()),
                float(sem.ae_grad(pool, p, idx=eval_idx, loss_kind=max_loss)[0].item()))

    loss_pca = losses(params)
    # Adam on the max-error loss (the squared form of the fallback's L-inf
    # bound) with the library's gradient and Adam kernels
    train_steps = 3000
    _, t_train = clock(lambda: sem.ae_train(pool, params, steps=train_steps, batch=2048,
                                            lr=3e-5, seed=0, warmup=100, cosine=True,
                                            loss_kind=max_loss))
    loss_ft = losses(params)
    del pool
    fields = list(W.ae_fields(63.5, dev, dtype=torch.float32))
    e = fields[0].shape[0]
    points = e * 512
    raw_bytes = e * 4 * 512 * 4
    reps = max(3, args.steps // 8)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        out = fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / reps

    n_raw_pca = sem.ae_compress(fields, params_pca)["n_raw"]
    pk, comp_ms = timed(lambda: sem.ae_compress(fields, params))
    dec, decomp_ms = timed(lambda: sem.ae_decompress(pk, params))
    mod, modal_ms = timed(lambda: sem.modal_compress(fields, recon=True))
    n_raw = pk["n_raw"]
    n_raw_mod = int(mod["flags"].sum().item())
    ratio = raw_bytes / sem.compressed_bytes(e, n_raw)
    ratio_mod = raw_bytes / sem.compressed_bytes(e, n_raw_mod)
    # relative L-inf error per channel of the decompressed fields
    err = []
    for a, b in zip(fields, dec):
        gm = float(a.abs().max().item())
        err.append(float((a - b).abs().max().item()) / gm if gm > 0 else 0.0)
    # Q isosurface of the decompressed velocity against the original's
    x, y, z = W.ae_mesh(dev, dtype=torch.float32)
    q0, _, mm0 = sem.qcrit(x, y, z, *fields[:3])
    flat = q0.reshape(-1)
    gen = torch.Generator(device=dev).manual_seed(0)
    idx = torch.randint(0, flat.numel(), (1 << 20,), device=dev, generator=gen)
    iso = float(torch.quantile(flat[idx].double(), 0.9).item())
    r0 = sem.isosurface(x, y, z, q0, [iso], minmax=mm0, cases=True)
    agree = {}
    for name, vel in (("network", dec[:3]), ("modal", mod["recon"][:3])):
        q1, _, mm1 = sem.qcrit(x, y, z, *vel)
        r1 = sem.isosurface(x, y, z, q1, [iso], minmax=mm1, cases=True)
        t0_, t1_ = int(r0["tri_count"][0].item()), int(r1["tri_count"][0].item())
        mism = float((r0["cases"] != r1["cases"]).float().mean().item())
        agree[name] = {"triangles": t1_, "triangle_rel_diff": abs(t1_ - t0_) / max(t0_, 1),
                       "case_mismatch_frac": mism,
                       "q_rel_linf": float((q1 - q0).abs().max().item())
                       / float(q0.abs().max().item())}
        del q1, r1
    tri0 = int(r0["tri_count"][0].item())
    log(args, f"compression: pool {t_pool:.1f} s, PCA init {t_pca * 1e3:.0f} ms, {train_steps} "
              f"Adam steps {t_train * 1e3:.0f} ms (max-error loss {loss_pca[1]:.3e} -> "
              f"{loss_ft[1]:.3e}; raw fallback of the PCA network {n_raw_pca / e:.4f}); compress "
              f"{comp_ms:.2f} ms ({points / (comp_ms * 1e-3) / 1e9:.1f} G points/s), "
              f"decompress {decomp_ms:.2f} ms; raw fallback {n_raw / e:.4f} (modal "
              f"{n_raw_mod / e:.4f}); ratio {ratio:.1f}x (modal {ratio_mod:.2f}x); Q "
              f"triangles {tri0} vs network {agree['network']['triangles']}, modal "
              f"{agree['modal']['triangles']}")
    out = {"elements": e, "points": points, "raw_bytes": raw_bytes,
           "pool_elements": 16384, "pca_init_ms": round(t_pca * 1e3, 2),
           "train_steps": train_steps, "train_batch": 2048,
           "train_ms": round(t_train * 1e3, 2),
           "train_loss": "max-error (mean squared per-(block, channel) maximum error), Adam "
                         "lr 3e-5, 100 warm-up steps, cosine decay",
           "mse_pca": loss_pca[0], "mse_trained": loss_ft[0],
           "max_loss_pca": loss_pca[1], "max_loss_trained": loss_ft[1],
           "pca_fallback_frac": n_raw_pca / e,
           "pca_ratio": raw_bytes / sem.compressed_bytes(e, n_raw_pca),
           "compress_ms": round(comp_ms, 4), "decompress_ms": round(decomp_ms, 4),
           "compress_points_per_s": points / (comp_ms * 1e-3),
           # one read of the four FP32 fields; latent, scales, flags and raw
           # elements written
           "compress_hbm": _hbm(raw_bytes + e * 81 + n_raw * 8192, comp_ms),
           # the linear network runs with layers 0-1 and 4-5 folded: 589,824
           # FLOPs per element (encoder 294,912, decoder 294,912) on FP32
           # matrix cores (and layers 2, 3 on the vector units)
           "compress_mfma": {"flops_per_element": 589824,
                             "achieved_tflops": round(589824 * e / (comp_ms * 1e-3) / 1e12, 2),
                             "peak_tflops": 157.3,
                             "frac": 589824 * e / (comp_ms * 1e-3) / 1e12 / 157.3},
           "modal_ms": round(modal_ms, 4),
           "fallback_frac": n_raw / e, "ratio": ratio,
           "modal_fallback_frac": n_raw_mod / e, "modal_ratio": ratio_mod,
           "rel_linf_per_channel": err, "q_isovalue": iso, "q_triangles": tri0,
           "isosurface_agreement": agree}
    del fields, dec, mod, pk, x, y, z, q0, r0
    torch.cuda.empty_cache()
    return out


def batched_timing(args, sem):
    """16 uneven FP32 snapshots (orders 5/7/9, 4,096-200,000 elements,
    stretched boxes; velocity plus a random-Fourier-feature scalar theta).
    Times: sem_qcrit per snapshot (16 launches) against sem_qcrit_batch (one
    persistent launch per order: with the default forms, then with the
    autotuned ones); and the whole step -- batched Q, then the
    isosurfaces of Q, |omega| and theta at 4 isovalues each per snapshot in
    one batched isosurface call (persistent count and emission kernels per
    order, one scan) -- eager and replayed as one captured HIP graph, beside
    the same step with 48 separate isosurface calls."""
    import torch

    import workloads as W
    dev = "cuda:0"
    t0 = time.time()
    snaps, theta, specs = [], [], []
    for seed in range(16):
        spec, arrs = W.batch_snapshot(seed, dev, dtype=torch.float32)
        x, y, z, u, v, w, th = arrs
        e = x.shape[0]
        snaps.append({"x": x, "y": y, "z": z, "u": u, "v": v, "w": w,
                      "q": torch.empty_like(u), "omega_mag": torch.empty_like(u),
                      "minmax": torch.empty((e, 2), dtype=torch.float32, device=dev)})
        theta.append(th)
        specs.append(spec)
    torch.cuda.synchronize()
    points = sum(sn["x"].numel() for sn in snaps)
    log(args, f"batched: 16 snapshots, {points} points generated in {time.time() - t0:.1f} s")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = max(3, args.steps // 4)
    # default forms (those of sem_qcrit), then the autotuned ones
    plan_default = sem.BatchPlan(snaps)
    default_variants = {n: sem.batch_variant(n, sem.SEM_F32) for n in (5, 7, 9)}
    tuned = {}
    for n in (5, 7, 9):
        var, ms = sem.autotune(n, sem.SEM_F32)
        tuned[n] = {"variant": var, "ms_variants": [round(m, 4) for m in ms]}
    plan = sem.BatchPlan(snaps)

    def per_snapshot():
        for sn in snaps:
            sem.qcrit(sn["x"], sn["y"], sn["z"], sn["u"], sn["v"], sn["w"], q=sn["q"],
                      omega_mag=sn["omega_mag"], minmax=sn["minmax"])

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    per_ms = timed(per_snapshot)
    default_ms = timed(lambda: sem.qcrit_batch(plan_default))
    batch_ms = timed(lambda: sem.qcrit_batch(plan))
    # isovalues of each field: quantiles 0.9 / 0.95 / 0.99 / 0.999 of a sample
    gen = torch.Generator(device=dev).manual_seed(0)
    isos, work = [], []
    sem.qcrit_batch(plan)
    for sn, th in zip(snaps, theta):
        per = []
        for f in (sn["q"], sn["omega_mag"], th):
            flat = f.reshape(-1)
            idx = torch.randint(0, flat.numel(), (1 << 20,), device=dev, generator=gen)
            qs = torch.quantile(flat[idx].double(), torch.tensor(
                [0.9, 0.95, 0.99, 0.999], dtype=torch.float64, device=dev))
            iv = [float(c) for c in qs.cpu()]
            r = sem.isosurface(sn["x"], sn["y"], sn["z"], f, iv)
            cap = int(r["tri_count"].sum().item())
            e = sn["x"].shape[0]
            ws = torch.empty(max(sem.workspace_bytes(e, sn["x"].shape[1] - 1, 4), 1),
                             dtype=torch.uint8, device=dev)
            per.append((f, iv, torch.empty((max(cap, 1), 3, 3), dtype=torch.float32,
                                           device=dev),
                        torch.zeros(4, dtype=torch.int64, device=dev), ws))
        isos.append(per)
    total_tri = sum(int(t[2].shape[0]) for per in isos for t in per)

    def step_per_call():
        sem.qcrit_batch(plan)
        for sn, per in zip(snaps, isos):
            for f, iv, tri, cnt, ws in per:
                sem.isosurface_into(sn["x"], sn["y"], sn["z"], f, iv, tri, cnt, ws)

    # the same 48 isosurfaces as one batched call: persistent count, one
    # scan, persistent emission
    jobs = []
    for i, (sn, per) in enumerate(zip(snaps, isos)):
        for (f, iv, _, _, _), name in zip(per, ("q", "omega_mag", None)):
            jobs.append({"snap": i, "field": name if name else f, "isovalues": iv})
    iso_plan = sem.IsoBatchPlan(snaps, jobs)
    b_tri = torch.empty((max(total_tri, 1), 3, 3), dtype=torch.float32, device=dev)
    b_cnt = torch.zeros(4 * len(jobs), dtype=torch.int64, device=dev)
    b_off = torch.zeros_like(b_cnt)

    def step():
        sem.qcrit_batch(plan)
        sem.isosurface_batch_into(iso_plan, b_tri, b_cnt, b_off)

    def graph_of(fn):
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        return g

    percall_eager_ms = timed(step_per_call)
    g_percall = graph_of(step_per_call)
    percall_graph_ms = timed(g_percall.replay)
    del g_percall
    eager_ms = timed(step)
    g = graph_of(step)
    graph_ms = timed(g.replay)
    # isosurface phase alone (Q already computed)
    iso_ms = timed(lambda: sem.isosurface_batch_into(iso_plan, b_tri, b_cnt, b_off))
    assert int(b_cnt.sum().item()) == total_tri
    log(args, f"batched: sem_qcrit x16 {per_ms:.3f} ms, sem_qcrit_batch default forms "
              f"{default_ms:.3f} ms, tuned {batch_ms:.3f} ms "
              f"({points / (batch_ms * 1e-3) / 1e9:.1f} G points/s); whole step (Q batch + "
              f"batched isosurfaces) eager {eager_ms:.3f} ms, graph {graph_ms:.3f} ms; "
              f"with 48 isosurface calls eager {percall_eager_ms:.3f} ms, graph "
              f"{percall_graph_ms:.3f} ms; variants "
              f"{({n: t['variant'] for n, t in tuned.items()})}")
    out = {"snapshots": 16, "points": points,
           "orders": [sp[0] for sp in specs], "elements": [sp[1][0] * sp[1][1] * sp[1][2]
                                                           for sp in specs],
           "default_variants": default_variants, "tuned": tuned,
           "qcrit_per_snapshot_ms": round(per_ms, 4),
           "qcrit_batch_default_ms": round(default_ms, 4),
           "qcrit_batch_ms": round(batch_ms, 4),
           "qcrit_batch_points_per_s": points / (batch_ms * 1e-3),
           # six FP32 inputs, Q and |omega| out, two range values per element
           "qcrit_batch_hbm": _hbm(32 * points + 8 * sum(
               sp[1][0] * sp[1][1] * sp[1][2] for sp in specs), batch_ms),
           "step_eager_ms": round(eager_ms, 4), "step_graph_ms": round(graph_ms, 4),
           "step_graph_points_per_s": points / (graph_ms * 1e-3),
           "isosurface_batch_ms": round(iso_ms, 4),
           "step_launches": "Q: one persistent kernel per order; isosurfaces: one persistent "
                            "count kernel per order, one scan (3 kernels + totals), one "
                            "persistent emission kernel per order",
           "step_per_call_eager_ms": round(percall_eager_ms, 4),
           "step_per_call_graph_ms": round(percall_graph_ms, 4),
           "triangles": total_tri}
    del snaps, theta, isos, plan, plan_default, g, iso_plan, b_tri
    torch.cuda.empty_cache()
    out["small"] = batched_small(args, sem, timed)
    return out


def batched_small(args, sem, timed):
    """256 small FP32 snapshots (orders 5/7/9, 64-2,048 elements each):
    where launches dominate, sem_qcrit per snapshot (256 launches) against
    sem_qcrit_batch (one launch per order), eager and replayed as a graph."""
    import torch

    import workloads as W
    dev = "cuda:0"
    snaps = []
    for seed in range(1000, 1256):
        _, arrs = W.batch_snapshot(seed, dev, dtype=torch.float32, features=16, e_min=64,
                                   e_max=2048)
        x, y, z, u, v, w, _ = arrs
        snaps.append({"x": x, "y": y, "z": z, "u": u, "v": v, "w": w,
                      "q": torch.empty_like(u), "omega_mag": torch.empty_like(u),
                      "minmax": torch.empty((x.shape[0], 2), dtype=torch.float32, device=dev)})
    torch.cuda.synchronize()
    points = sum(sn["x"].numel() for sn in snaps)
    plan = sem.BatchPlan(snaps)

    def per_snapshot():
        for sn in snaps:
            sem.qcrit(sn["x"], sn["y"], sn["z"], sn["u"], sn["v"], sn["w"], q=sn["q"],
                      omega_mag=sn["omega_mag"], minmax=sn["minmax"])

    per_ms = timed(per_snapshot)
    batch_ms = timed(lambda: sem.qcrit_batch(plan))
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            sem.qcrit_batch(plan)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph_ms = timed(g.replay)
    log(args, f"batched small: 256 snapshots, {points} points: sem_qcrit x256 {per_ms:.3f} ms, "
              f"sem_qcrit_batch {batch_ms:.3f} ms, graph {graph_ms:.3f} ms")
    out = {"snapshots": 256, "points": points, "qcrit_per_snapshot_ms": round(per_ms, 4),
           "qcrit_batch_ms": round(batch_ms, 4), "qcrit_batch_graph_ms": round(graph_ms, 4),
           "qcrit_batch_graph_points_per_s": points / (graph_ms * 1e-3)}
    del snaps, plan, g
    torch.cuda.empty_cache()
    return out


def c0_timing(args, sem, fields, q, isos, n):
    """C0 averaging of Q over the shared GLL nodes (sem_dsavg with a
    gather-scatter built once by sem_gs_setup), the isosurfaces of the
    averaged Q with edge keys, their global keys, and welding."""
    import torch

    import workloads as W
    dev = q.device
    gid = torch.from_numpy(W.lattice_gid(W.CHANNEL_SHAPE, n)).to(dev)
    n_glob = 1
    for s_ax in W.CHANNEL_SHAPE:
        n_glob *= s_ax * n + 1                  # lattice points of the box mesh
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # the first build also allocates the workspace (and finds the node count
    # from the ids, a device reduction and a host sync); a mesh's setup is
    # timed on the second build, with the node count given
    torch.cuda.synchronize()
    t0 = time.time()
    gs = sem.GatherScatter(gid)
    torch.cuda.synchronize()
    first_ms = (time.time() - t0) * 1e3
    assert gs.n_global == n_glob
    del gs
    torch.cuda.synchronize()
    e0.record()
    gs = sem.GatherScatter(gid, n_global=n_glob)
    e1.record()
    torch.cuda.synchronize()
    setup_ms = e0.elapsed_time(e1)
    qa = torch.empty_like(q)
    reps = max(3, args.steps // 4)
    sem.dsavg(q, gs, out=qa)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        sem.dsavg(q, gs, out=qa)
    e1.record()
    torch.cuda.synchronize()
    avg_ms = e0.elapsed_time(e1) / reps
    x, y, z = fields[:3]
    r = sem.isosurface(x, y, z, qa, isos, edge_keys=True)
    keys = sem.global_edge_keys(r["edge_key"], gid)
    sem.weld(r["tri_xyz"], keys)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        keys = sem.global_edge_keys(r["edge_key"], gid)
        verts, idx = sem.weld(r["tri_xyz"], keys)
    e1.record()
    torch.cuda.synchronize()
    weld_ms = e0.elapsed_time(e1) / reps
    n_tri = int(r["tri_xyz"].shape[0])
    log(args, f"C0: gather-scatter setup {setup_ms:.3f} ms (first build, with its "
              f"allocation, {first_ms:.1f} ms), dsavg {avg_ms:.4f} ms, "
              f"global keys + weld {weld_ms:.4f} ms: {n_tri} triangles -> "
              f"{int(verts.shape[0])} vertices")
    n_global = gs.n_global
    n_nodes = int(q.numel())
    del gid, gs, qa
    # dsavg: row pointers, column list, field in and out (FP64)
    dbytes = 8 * (n_global + 1) + 24 * n_nodes
    return {"gs_setup_ms": round(setup_ms, 4), "gs_setup_first_ms": round(first_ms, 3),
            "dsavg_ms": round(avg_ms, 5),
            "keys_weld_ms": round(weld_ms, 5), "triangles": n_tri,
            "welded_vertices": int(verts.shape[0]), "n_global": n_global,
            "dsavg_hbm": _hbm(dbytes, avg_ms)}


def _hbm(nbytes, ms):
    """Algorithmic bytes of one call against the 8 TB/s HBM peak."""
    gbps = nbytes / (ms * 1e-3) / 1e9
    return {"bytes": int(nbytes), "achieved_gbps": round(gbps, 1), "peak_gbps": 8000.0,
            "frac": round(gbps / 8000.0, 4)}


def precision_modes(args, sem, fields, isos, n_elem, points):
    """The same sem_extract step in FP32 storage: plain FP32 and the mixed
    modes (BF16 / FP16 matrix-core contractions, plain and split).  Returns
    {mode: {ms_per_step, points_per_s, q_phase_ms, triangles}}."""
    import torch
    f32 = [f.float().contiguous() for f in fields]
    k = len(isos)
    mfma = measured_mfma()
    dev = f32[0].device
    out = {}
    for mode in ("f32", "bf16", "fp16", "bf16x3", "fp16x3"):
        prec = None if mode == "f32" else mode
        code = sem.SEM_F32 if prec is None else sem.MIXED[prec]
        ws = torch.empty(sem.extract_workspace_bytes(n_elem, 7, k, code), dtype=torch.uint8,
                         device=dev)
        cnt = torch.zeros(k, dtype=torch.int64, device=dev)
        sem.extract_into(*f32, isos, [None] * k, cnt, ws, precision=prec)
        counts = cnt.cpu().tolist()
        tris = [torch.empty((c, 3, 3), dtype=torch.float32, device=dev) for c in counts]
        q = torch.empty_like(f32[3])
        om = torch.empty_like(f32[3])
        mm = torch.empty((n_elem, 2), dtype=torch.float32, device=dev)

        def step():
            sem.extract_into(*f32, isos, tris, cnt, ws, q=q, omega_mag=om, minmax=mm,
                             precision=prec)

        for _ in range(2):
            step()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        steps = max(5, args.steps // 2)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        sem.timing_begin(4 * steps + 16)
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ph, _ = sem.timing_end()
        qms = ph["qcrit"][0] / max(ph["qcrit"][1], 1)
        out[mode] = {"ms_per_step": round(ms, 5), "points_per_s": points / (ms * 1e-3),
                     "q_phase_ms": round(qms, 5), "triangles": counts}
        flops = mfma.get(mode)
        if flops:
            ach = flops / (qms * 1e-3) / 1e12
            out[mode]["mfma"] = {"flops_per_launch": flops, "achieved_tflops": round(ach, 2),
                                 "peak_tflops": MFMA_PEAK_TFLOPS,
                                 "frac": round(ach / MFMA_PEAK_TFLOPS, 5)}
        log(args, f"{mode:7s}: {ms:.4f} ms/step ({points / (ms * 1e-3) / 1e9:.1f} G points/s), "
                  f"Q phase {qms:.4f} ms, triangles {counts}")
        del ws, tris, q, om, mm
    return out


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
    # the elements are independent: worker threads take chunks of 512
    # elements each (numpy releases the interpreter lock inside its array
    # operations), with BLAS held to one thread per worker, so `cores` is
    # the number of threads actually computing
    import concurrent.futures
    from threadpoolctl import threadpool_limits
    workers = max(1, min(16, os.cpu_count() or 1))
    chunk = 512

    def work(a0):
        sl = slice(a0, min(a0 + chunk, k))
        part = [a[sl] for a in arrs]
        q, _, _ = osem.qcrit(*part, d)
        mc.extract(*part[:3], q, isos)

    with threadpool_limits(1):
        t0 = time.perf_counter()
        with concurrent.futures.ThreadPoolExecutor(workers) as ex:
            list(ex.map(work, range(0, k, chunk)))
        dt_s = time.perf_counter() - t0
    pts = k * (n + 1) ** 3
    log(args, f"cpu oracle: {k} elements in {dt_s:.2f} s with {workers} worker threads")
    return {"value": pts / dt_s, "unit": "GLL points/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{k} random elements of the same snapshot ({pts} points), "
                      f"FP64 numpy oracle, Q + |omega| + {len(isos)} isosurfaces, "
                      f"chunks of {chunk} elements on {workers} threads (BLAS one thread "
                      f"each), {dt_s:.2f} s wall"}


def _csv(directory, suffix):
    import csv
    import glob
    found = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not found:
        sys.exit(f"no *{suffix} under {directory}")
    with open(found[0]) as fh:
        return list(csv.DictReader(fh))


def _short(name):
    name = name.replace("sem::(anonymous namespace)::", "")
    return name.split("(")[0] if not name.startswith("void ") else name[5:].split("(")[0]


def summarize_trace(directory, out, command):
    """Text table of a rocprofv3 --kernel-trace --stats run (library kernels,
    the copy kernel; torch's input-generation kernels summed in one line)."""
    rows = _csv(directory, "kernel_stats.csv")
    lines = [f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_ms':>9}  kernel"]
    other = [0, 0.0]
    for r in rows:
        name = r["Name"]
        if "at::native" in name:
            other[0] += int(r["Calls"])
            other[1] += float(r["TotalDurationNs"]) / 1e6
            continue
        lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:9.3f}  {_short(name)}")
    lines.append(f"{other[0]:6d} {'':10} {'':10} {'':10} {other[1]:9.3f}  "
                 "(torch kernels: synthetic input generation)")
    with open(out, "w") as fh:
        fh.write(f"# rocprofv3 kernel trace, MI355X\n# command: {command}\n"
                 f"# kernel source sha256: {kernel_sha()}\n\n" + "\n".join(lines) + "\n")
    print(open(out).read())


def summarize_mfma(directory, out, command):
    """Matrix-core work per launch of the mixed-precision Q kernels
    (mixed7<mode, true, true>, sem_extract): SQ_INSTS_VALU_MFMA_MOPS_BF16 /
    _F16 count matrix operations in units of 512 FLOPs."""
    per = {}
    for r in _csv(directory, "counter_collection.csv"):
        name = _short(r["Kernel_Name"])
        if not name.startswith("mixed7<") or not name.endswith("true, true>"):
            continue
        mode = MIX_MODES.get(name[len("mixed7<"):].split(",")[0].strip())
        if mode is None:
            continue
        per.setdefault(mode, {}).setdefault(r["Counter_Name"], []).append(
            float(r["Counter_Value"]))
    modes = {}
    for mode, ctr in per.items():
        avg = {k: sum(v) / len(v) for k, v in ctr.items()}
        mops = avg.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) + avg.get(
            "SQ_INSTS_VALU_MFMA_MOPS_F16", 0.0)
        modes[mode] = {"dispatches": len(next(iter(ctr.values()))),
                       "counters_per_dispatch": avg,
                       "mfma_flops_per_launch": mops * 512.0}
    rec = {"kernel": "mixed7<mode, true, true>",
           "workload": "channel 65,536 order-7 elements, 3 Q isovalues, FP32 storage",
           "kernel_src_sha256": kernel_sha(), "command": command, "modes": modes}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def summarize_pmc(fetch_dir, write_dir, out, command):
    """HBM bytes per dispatch of the Q kernel from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by what the counter reads for the 1 GiB
    calibration copy of the same run (a plain copy kernel of known traffic).
    Writes the JSON `measured_traffic` reads."""
    import numpy as np
    res = {}
    for counter, directory in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = {}
        for r in _csv(directory, "counter_collection.csv"):
            if r["Counter_Name"] != counter:
                continue
            per.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        # the run's 1 GiB copies (the calibration call and the bandwidth
        # reps; the 512 MiB cache flushes read about half as much): the
        # median counter value of one such dispatch
        copies = per.get("stream_copy16", [])
        top = max(copies)
        one = sorted(v for v in copies if v > 0.75 * top)
        scale = CALIBRATION_BYTES / (one[len(one) // 2] * 1024.0)
        res[counter] = (per, scale)
    dtype = "f64" if "f64" in os.path.basename(out) else "f32"
    kname = q_kernel_name(dtype)
    fetch = float(np.mean(res["FETCH_SIZE"][0][kname]))
    write = float(np.mean(res["WRITE_SIZE"][0][kname]))
    fs, wsc = res["FETCH_SIZE"][1], res["WRITE_SIZE"][1]
    rec = {
        "kernel": kname,
        "workload": "channel 65,536 order-7 elements, 3 Q isovalues, " + dtype,
        "kernel_src_sha256": kernel_sha(),
        "points_per_launch": 65536 * 512,
        "dispatches": len(res["FETCH_SIZE"][0][kname]),
        "fetch_kib_per_dispatch": fetch,
        "write_kib_per_dispatch": write,
        "fetch_scale": round(fs, 4),
        "write_scale": round(wsc, 4),
        "hbm_read_bytes_per_launch": int(fetch * 1024 * fs),
        "hbm_write_bytes_per_launch": int(write * 1024 * wsc),
        "hbm_bytes_per_launch": int(fetch * 1024 * fs + write * 1024 * wsc),
        "command": command,
        "other_kernels_kib_per_dispatch": {
            k: {"fetch": float(np.mean(v)),
                "write": float(np.mean(res["WRITE_SIZE"][0].get(k, [0.0])))}
            for k, v in res["FETCH_SIZE"][0].items() if "at::native" not in k},
    }
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
