"""Benchmark of the 3D DRT hot path on one MI355X.

Workload: the 3D DRT of planes of one N=512 int32 cube over all 12 dodecants,
a sparse point cloud (1% occupancy, value 1) plus 8 planes with random normals
(value 16), seed 2. A step is one drt3d_forward call (frame transposes and
every fused stage pass); the input is resident in HBM before timing starts.

Prints one JSON line. `value` is voxel-stage updates per second,
U = 12 * log2(N) * N^2 * 3N (Algorithm 1's writes per stage, summed over the
stages and dodecants). `roofline` covers the dominant kernel, timed with HIP
events recorded on the launch stream around every launch of the timed
region; its algorithmic bytes are the reads of each pass's input extent plus
the writes of its output extent. `cpu_baseline` times the oracle's naive
Algorithm 1 on one dodecant of the same cube (scaled to the job).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def updates(N, ndod=12):
    n = N.bit_length() - 1
    return ndod * n * N * N * 3 * N


def _traffic_record(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    import hashlib
    src = os.path.join(ROOT, "paper_2501_13664_amd", "csrc", "drt3d_device.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    ent = rec.get(kernel)
    if not ent or ent.get("source_sha256") != h:
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(vol):
    import oracle
    N = vol.shape[0]
    t0 = time.perf_counter()
    oracle.rec_drt(vol, 0x001)
    dt = time.perf_counter() - t0
    return {
        "value": updates(N, 1) / dt,
        "unit": "voxel-stage updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "dodecant 0 of the same N=%d cube (1/12 of the job), naive Algorithm 1 on "
                  "full-extent int64 buffers, one thread: %.2f s" % (N, dt),
    }


def batched_speedup(api, torch, reps=5):
    """96 float32 cubes of mixed N: one batched call vs per-volume calls."""
    import workloads
    cubes = [torch.from_numpy(c).cuda() for c in workloads.mixed_batch()]
    outs = [torch.empty(api.drt3d_out_shape(c.shape[0]), dtype=torch.float32, device="cuda") for c in cubes]
    ws_b = None
    api.drt3d_forward_batched(cubes, outs=outs)
    torch.cuda.synchronize()

    def per_volume():
        for c, o in zip(cubes, outs):
            api.drt3d_forward(c, out=o)

    def batched():
        api.drt3d_forward_batched(cubes, outs=outs, workspace=ws_b)

    res = {}
    for name, fn in (("per_volume", per_volume), ("batched", batched)):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        res[name] = best * 1e3
    U = sum(updates(c.shape[0]) for c in cubes)
    return {"per_volume_ms": res["per_volume"], "batched_ms": res["batched"],
            "speedup": res["per_volume"] / res["batched"], "updates": U,
            "batched_updates_per_s": U / (res["batched"] / 1e3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2501_13664_amd import api

    N = args.N
    vol_np = workloads.point_cloud_with_planes(N, seed=2)
    vol = torch.from_numpy(vol_np).cuda()
    out = torch.empty(api.drt3d_out_shape(N), dtype=torch.int32, device="cuda")
    from paper_2501_13664_amd._lib import lib
    ws = torch.empty(lib().drt3d_workspace_bytes(N, 0xFFF, 0), dtype=torch.uint8, device="cuda")

    for _ in range(args.warmup):
        api.drt3d_forward(vol, out=out, workspace=ws)
    torch.cuda.synchronize()

    with api.profile() as prof:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            api.drt3d_forward(vol, out=out, workspace=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    U = updates(N)
    value = U / (ms / 1e3)

    # dominant kernel by summed time
    recs = prof.records
    dom = max(recs, key=lambda k: recs[k][0])
    dms, dn, dbytes = recs[dom]
    per_launch_ms = dms / dn
    achieved = (dbytes / dn) / (per_launch_ms / 1e3) / 1e9
    kernels = {k: {"ms_total": v[0], "launches": v[1], "ms_per_launch": v[0] / v[1],
                   "alg_GBps": (v[2] / v[1]) / (v[0] / v[1] / 1e3) / 1e9} for k, v in recs.items()}
    total_alg = sum(v[2] for v in recs.values())
    total_ms = sum(v[0] for v in recs.values())

    line = {
        "metric": "3D DRT N=512 voxel-stage updates/s + HBM GB/s %peak; batched vs per-volume speedup",
        "value": value,
        "unit": "voxel-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "drt3d_forward N=%d int32, 12 dodecants, 1%% point cloud + 8 planes (seed 2)" % N,
                   "N": N, "dodecants": 12, "parallelism": "single-gpu"},
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": _traffic_record(dom),
        },
        "hbm_alg_GBps_all_kernels": total_alg / (total_ms / 1e3) / 1e9,
        "kernels": kernels,
    }
    if not args.no_batched:
        line["batched_vs_per_volume"] = batched_speedup(api, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(vol_np)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
