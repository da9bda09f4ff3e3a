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
the writes of its output extent; `traffic` is the HBM bytes per launch from
the committed rocprofv3 counter summary when it was taken on the current
sources. `compulsory_floor` relates the time per transform to the least HBM
traffic any implementation needs (read the volume once per dodecant, write the
output once) at the 8 TB/s peak. `cpu_baseline` times the oracle's naive
Algorithm 1 on the same cube on the host: one thread on one dodecant, and all
12 dodecants on parallel threads (the whole job); that leg, the only one that
runs the oracle, also measures each float32 result of the batched and
differentiable legs against the FP64 oracle (normwise error and
max |err| / R(|f|), written into those legs as `fp64_error`).

Further measurements ride along (skipped with --no-adjoint / --no-batched /
--no-diff / --no-djt / --no-inverse): the adjoint of the benchmark's
projections; the batched forward of 96 float32 cubes of mixed N against
per-volume calls; the differentiable transform (forward + backward through
autograd) of a batch of 8 float32 N=128 cubes against per-volume forward +
adjoint calls (both check that the two ways give bit-identical results); the
3D DJT of one N=128 int32 cube, with U = 12 * 8 N^3 (N-1) voxel-stage updates,
and its adjoint; Algorithm 2's merged net of the projections and the same cube's
forward as uint8 with narrow storage (both with the adjoint); the
iterative inverse of a float32 N=128 DRT (ten V-cycles) with its error after
each cycle count; and plane detection (Sec. 6.1, --no-planes): on the
benchmark's projections, and end to end (forward, detection, backprojection)
on an N=128 voxelized room scene.

--copy-calibration runs only a plain 1 GiB device-to-device copy (five times),
the reference kernel that scales the HBM byte counters.
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


def floor_record(N, ms):
    """The transform's compulsory HBM traffic (read the input once per
    dodecant, write the 12 N^2 (3N-2) int32 output once), its time at the 8 TB/s
    peak, and the measured time per transform as a multiple of it."""
    nbytes = 12 * 4.0 * N ** 3 + 12 * 4.0 * N * N * (3 * N - 2)
    floor_ms = nbytes / (HBM_PEAK_GBS * 1e9) * 1e3
    return {"bytes": nbytes, "floor_ms": floor_ms, "ms_per_transform": ms, "ratio_to_floor": ms / floor_ms}


def updates(N, ndod=12):
    n = N.bit_length() - 1
    return ndod * n * N * N * 3 * N


CSRC = "paper_2501_13664_amd/csrc"


def sources_sha256():
    """One hash over every HIP source and header of the library (kernels and
    launch planning), in name order: a counter record taken on other sources
    no longer describes the kernels that run."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, CSRC)
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()


def _traffic_record(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = rec.get(kernel)
    if not ent or ent.get("sources_sha256") != sources_sha256():
        return None
    return ent.get("bytes_per_launch")


def _host_info():
    """Host CPU model and thread counts as the GPU machine's own host reports them."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    if model is None:
        try:
            import subprocess
            out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
            model = next((l.split(":", 1)[1].strip() for l in out.splitlines() if l.startswith("Model name")), None)
        except OSError:
            pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    avail = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemAvailable:"):
                avail = int(line.split()[1]) * 1024
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "affinity": affinity, "mem_available_bytes": avail}


def _fp64_errors(y32, y64, r_abs):
    """Normwise relative L2 error of a float32 result against FP64, and the
    largest |y32 - y64| / R(|f|) (R(|f|): the same transform of |f| in FP64)."""
    y32 = np.asarray(y32, dtype=np.float64)
    d = y32 - y64
    nw = float(np.linalg.norm(d) / max(np.linalg.norm(y64), 1e-300))
    m = r_abs > 0
    mx = float(np.max(np.abs(d[m]) / r_abs[m])) if m.any() else 0.0
    if (~m).any():
        mx = max(mx, float("inf") if np.any(d[~m] != 0) else 0.0)
    return nw, mx


def cpu_baseline(vol, float_checks=()):
    """The oracle on the GPU machine's host cores: its naive Algorithm 1 on the
    N=512 benchmark cube, once on one thread for dodecant 0 and once for all 12
    dodecants on parallel threads (one dodecant per thread; the oracle's C
    calls release the GIL), so `value` is the whole job's rate on `cores`
    threads.

    This leg is also where the float legs' results meet the FP64 oracle (the
    only part of the benchmark that runs it): each entry of float_checks is
    (leg dict, name, float32 result, kind, input, N) and gets its normwise
    error and max |err| / R(|f|) written into leg["fp64_error"][name]."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    N = vol.shape[0]
    host = _host_info()
    t0 = time.perf_counter()
    oracle.rec_drt(vol, 0x001)
    t1 = time.perf_counter() - t0
    # one dodecant holds about 4 N^2 (3N) int64 cells of buffers and output
    per_thread = 4 * N * N * 3 * N * 8
    threads = min(12, host["affinity"] or 1, 16)
    if host["mem_available_bytes"]:
        threads = max(1, min(threads, int(0.6 * host["mem_available_bytes"] // per_thread)))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda k: oracle.rec_drt(vol, 1 << k).shape, range(12)))
    tp = time.perf_counter() - t0
    res = {
        "value": updates(N, 12) / tp,
        "unit": "voxel-stage updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "the whole job: all 12 dodecants of the same N=%d cube, naive Algorithm 1 on full-extent "
                  "int64 buffers, one dodecant per thread on %d threads: %.2f s; one thread on dodecant 0: "
                  "%.2f s" % (N, threads, tp, t1),
        "one_thread": {"value": updates(N, 1) / t1, "seconds_one_dodecant": t1},
        "parallel": {"threads": threads, "seconds_12_dodecants": tp, "value": updates(N, 12) / tp},
        "host": host,
    }
    t0 = time.perf_counter()

    def check(item):
        leg, name, y32, kind, inp, Nc = item
        x64 = np.asarray(inp, dtype=np.float64)
        if kind == "drt":
            y64, r = oracle.rec_drt(x64), oracle.rec_drt(np.abs(x64))
        else:  # the adjoint of a projection
            y64, r = oracle.rec_adj(x64, Nc), oracle.rec_adj(np.abs(x64), Nc)
        return leg, name, _fp64_errors(y32, y64, r)

    items = list(float_checks)
    with ThreadPoolExecutor(max_workers=max(1, min(8, host["affinity"] or 1))) as ex:
        for leg, name, (nw, mx) in ex.map(check, items):
            e = leg.setdefault("fp64_error", {"tolerance": 1e-5, "results": {}})
            e["results"][name] = {"normwise": nw, "max_over_R_abs_f": mx}
            e["worst_normwise"] = max(e.get("worst_normwise", 0.0), nw)
            e["worst_max_over_R_abs_f"] = max(e.get("worst_max_over_R_abs_f", 0.0), mx)
    if items:
        res["fp64_checks_seconds"] = time.perf_counter() - t0
    return res


def _best_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best * 1e3


def call_roofline(api, torch, fn, ms):
    """HBM roofline of a whole call: the algorithmic bytes of every library
    launch it makes (one profiled run) over the call's best wall time."""
    with api.profile() as prof:
        fn()
        torch.cuda.synchronize()
    nbytes = sum(v[2] for v in prof.records.values())
    kernel_ms = sum(v[0] for v in prof.records.values())
    achieved = nbytes / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "bytes_per_call": nbytes, "kernel_ms": kernel_ms,
            "launches": sum(v[1] for v in prof.records.values())}


def batched_speedup(api, torch, reps=5):
    """96 float32 cubes of mixed N (48 x 32^3, 32 x 64^3, 12 x 128^3, 4 x 256^3):
    one batched call vs per-volume calls on the same stream."""
    import workloads
    cubes = [torch.from_numpy(c).cuda() for c in workloads.mixed_batch()]
    outs = [torch.empty(api.drt3d_out_shape(c.shape[0]), dtype=torch.float32, device="cuda") for c in cubes]

    def per_volume():
        for c, o in zip(cubes, outs):
            api.drt3d_forward(c, out=o)

    def batched():
        api.drt3d_forward_batched(cubes, outs=outs)

    pv = _best_ms(torch, per_volume, reps)
    ref = [o.clone() for o in outs]
    bt = _best_ms(torch, batched, reps)
    same = all(torch.equal(a, b) for a, b in zip(ref, outs))
    del ref
    U = sum(updates(c.shape[0]) for c in cubes)
    leg = {"workload": "96 float32 N(0,1) cubes, seeds 1000+i: 48x32^3 + 32x64^3 + 12x128^3 + 4x256^3, "
                       "12 dodecants",
           "per_volume_ms": pv, "batched_ms": bt, "speedup": pv / bt, "bit_identical": same,
           "updates": U, "batched_updates_per_s": U / (bt / 1e3),
           "roofline": call_roofline(api, torch, batched, bt),
           "fp64_error_sample": "every output of all 48 N=32 and 32 N=64 cubes, of the first two N=128 cubes "
                                "and of the first N=256 cube"}
    # the batched call's results, for the FP64 comparison in the cpu_baseline leg
    seen = {}
    checks = []
    for i, (c, o) in enumerate(zip(workloads.mixed_batch(), outs)):
        Nc = c.shape[0]
        seen[Nc] = seen.get(Nc, 0) + 1
        if Nc <= 64 or (Nc == 128 and seen[Nc] <= 2) or (Nc == 256 and seen[Nc] <= 1):
            checks.append((leg, "cube%d_N%d" % (i, Nc), o.cpu().numpy(), "drt", c, Nc))
    return leg, checks


def differentiable_speedup(api, torch, reps=5):
    """Batch of 8 float32 N=128 cubes, 12 dodecants: forward + backward through
    the autograd Function (batched launches) vs per-volume forward + adjoint."""
    import workloads
    from paper_2501_13664_amd import autograd
    B, N = 8, 128
    f = torch.from_numpy(workloads.normal_batch(B, N, seed=5)).cuda()
    g = torch.from_numpy(workloads.normal_weights((B,) + api.drt3d_out_shape(N), seed=6)).cuda()
    y = torch.empty_like(g)
    x = torch.empty_like(f)

    def per_volume():
        for b in range(B):
            api.drt3d_forward(f[b], out=y[b])
            api.drt3d_adjoint(g[b], out=x[b])

    fr = f.clone().requires_grad_(True)
    state = {}

    def differentiable():
        fr.grad = None
        out = autograd.drt3d(fr)
        out.backward(g)
        state["y"] = out

    pv = _best_ms(torch, per_volume, reps)
    ad = _best_ms(torch, differentiable, reps)
    same = torch.equal(state["y"].detach(), y) and torch.equal(fr.grad, x)
    U = 2 * B * updates(N)
    leg = {"workload": "8 float32 N(0,1) cubes N=128 (seed 5), 12 dodecants, grad_out N(0,1) (seed 6)",
           "per_volume_ms": pv, "autograd_ms": ad, "speedup": pv / ad, "bit_identical": same,
           "updates": U, "autograd_updates_per_s": U / (ad / 1e3),
           "roofline": call_roofline(api, torch, differentiable, ad),
           "fp64_error_sample": "every output of cubes 0 and 1: the forward R f and the gradient R^T g"}
    f_np = workloads.normal_batch(B, N, seed=5)
    g_np = workloads.normal_weights((B,) + api.drt3d_out_shape(N), seed=6)
    checks = []
    for b in (0, 1):
        checks.append((leg, "forward_cube%d" % b, state["y"][b].detach().cpu().numpy(), "drt", f_np[b], N))
        checks.append((leg, "backward_cube%d" % b, fr.grad[b].cpu().numpy(), "adj", g_np[b], N))
    return leg, checks


def adjoint_rate(api, torch, proj, N, reps=3):
    """The DRT adjoint (backprojection) of the benchmark's own N=512 int32
    projections, all 12 dodecants: the same recursion run in reverse."""
    from paper_2501_13664_amd._lib import lib
    back = torch.empty((N, N, N), dtype=torch.int32, device="cuda")
    ws = torch.empty(lib().drt3d_adjoint_workspace_bytes(N, 0xFFF, 0), dtype=torch.uint8, device="cuda")
    api.drt3d_adjoint(proj, out=back, workspace=ws)
    torch.cuda.synchronize()
    with api.profile() as prof:
        ms = _best_ms(torch, lambda: api.drt3d_adjoint(proj, out=back, workspace=ws), reps)
    recs = prof.records
    dom = max(recs, key=lambda k: recs[k][0])
    dms, dn, dbytes = recs[dom]
    achieved = (dbytes / dn) / (dms / dn / 1e3) / 1e9
    U = updates(N)
    return {"workload": "drt3d_adjoint N=%d int32, 12 dodecants, of the forward's projections" % N,
            "ms": ms, "updates": U, "updates_per_s": U / (ms / 1e3),
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": dbytes / dn},
            "kernels": {k: {"ms_total": v[0], "launches": v[1], "alg_GBps": v[2] / (v[0] / 1e3) / 1e9}
                        for k, v in recs.items()}}


def djt_rate(api, torch, reps=3):
    """The 3D DJT of lines of one N=128 int32 cube (uniform noise in [0,3] plus
    64 segments of value 8, seed 3) over all 12 dodecants: 4D output
    12 x 128 x 128 x 255 x 255 (51 GB)."""
    import workloads
    N = 128
    vol = torch.from_numpy(workloads.noise_with_segments(N, seed=3)).cuda()
    out = torch.empty(api.djt3d_out_shape(N), dtype=torch.int32, device="cuda")
    from paper_2501_13664_amd._lib import lib
    ws = torch.empty(lib().djt3d_workspace_bytes(N, 0xFFF, 0), dtype=torch.uint8, device="cuda")
    api.djt3d_forward(vol, out=out, workspace=ws)
    torch.cuda.synchronize()
    with api.profile() as prof:
        ms = _best_ms(torch, lambda: api.djt3d_forward(vol, out=out, workspace=ws), reps)
    recs = prof.records
    dom = max(recs, key=lambda k: recs[k][0])
    dms, dn, dbytes = recs[dom]
    achieved = (dbytes / dn) / (dms / dn / 1e3) / 1e9
    U = 12 * 8 * N ** 3 * (N - 1)
    res = {"workload": "djt3d_forward N=128 int32, 12 dodecants, noise [0,3] + 64 segments (seed 3)",
           "ms": ms, "updates": U, "updates_per_s": U / (ms / 1e3),
           "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS},
           "kernels": {k: {"ms_total": v[0], "launches": v[1], "alg_GBps": v[2] / (v[0] / 1e3) / 1e9}
                       for k, v in recs.items()}}
    # the transpose, backprojecting that DJT output
    del ws
    ws = torch.empty(lib().djt3d_adjoint_workspace_bytes(N, 0xFFF, 0), dtype=torch.uint8, device="cuda")
    back = torch.empty((N, N, N), dtype=torch.int32, device="cuda")
    api.djt3d_adjoint(out, out=back, workspace=ws)
    torch.cuda.synchronize()
    with api.profile() as prof:
        ams = _best_ms(torch, lambda: api.djt3d_adjoint(out, out=back, workspace=ws), reps)
    recs = prof.records
    dom = max(recs, key=lambda k: recs[k][0])
    dms, dn, dbytes = recs[dom]
    achieved = (dbytes / dn) / (dms / dn / 1e3) / 1e9
    res["adjoint"] = {"workload": "djt3d_adjoint N=128 int32, 12 dodecants, of the forward's output",
                      "ms": ams, "updates_per_s": U / (ams / 1e3),
                      "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS},
                      "kernels": {k: {"ms_total": v[0], "launches": v[1], "alg_GBps": v[2] / (v[0] / 1e3) / 1e9}
                                  for k, v in recs.items()}}
    return res


def narrow_rate(api, torch, vol_np, ref, reps=5):
    """The same N=512 cube as uint8 (its values are 0, 1 and 16) through the
    narrow-storage forward: the identical int32 projections with fewer HBM
    bytes (1-byte volume copies, 16-bit first-stage partial sums)."""
    N = vol_np.shape[0]
    v8 = torch.from_numpy(vol_np.astype("uint8")).cuda()
    v32 = torch.from_numpy(vol_np).cuda()
    out = torch.empty_like(ref)
    from paper_2501_13664_amd._lib import lib
    ws = torch.empty(lib().drt3d_workspace_bytes(N, 0xFFF, 2), dtype=torch.uint8, device="cuda")
    ws32 = torch.empty(lib().drt3d_workspace_bytes(N, 0xFFF, 0), dtype=torch.uint8, device="cuda")
    # both forms timed the same way, back to back, outside the profiler
    ms32 = _best_ms(torch, lambda: api.drt3d_forward(v32, out=out, workspace=ws32), reps)
    ms = _best_ms(torch, lambda: api.drt3d_forward(v8, out=out, workspace=ws), reps)
    same = bool(torch.equal(out, ref))
    with api.profile() as prof:
        api.drt3d_forward(v8, out=out, workspace=ws)
        torch.cuda.synchronize()
    recs = prof.records
    U = updates(N)
    return {"workload": "drt3d_forward N=%d, the benchmark cube as uint8, int32 out, 12 dodecants" % N,
            "ms": ms, "int32_ms": ms32, "faster_than_int32": 1.0 - ms / ms32,
            "updates_per_s": U / (ms / 1e3), "bit_identical_to_int32": same,
            "kernels": {k: {"ms_per_launch": v[0] / v[1], "alg_GBps": v[2] / (v[0] / 1e3) / 1e9} for k, v in recs.items()}}


def merge_net_rate(api, torch, proj, reps=3):
    """Algorithm 2's merged net of the benchmark's N=512 projections: reads the
    12 dodecants once, writes the 4N x 4N x (3N-2) net once (corners zeroed)."""
    N = int(proj.shape[1])
    net = torch.empty((4 * N, 4 * N, 3 * N - 2), dtype=proj.dtype, device="cuda")
    ms = _best_ms(torch, lambda: api.drt3d_merge_net(proj, out=net), reps)
    nbytes = 4.0 * (12 + 16) * N * N * (3 * N - 2)
    del net
    return {"workload": "drt3d_merge_net N=%d int32 (the forward's projections)" % N, "ms": ms,
            "bytes": nbytes, "GBps": nbytes / (ms / 1e3) / 1e9, "frac_of_hbm_peak": nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}


def planes_rate(api, torch, proj, reps=3):
    """Plane detection (Sec. 6.1): on the benchmark's N=512 projections (the
    maximum reads all 19.3 GB once; the peak search reads the columns
    orthogonal to the dominant plane), and the whole application on a
    voxelized N=128 room scene: forward, detection, backprojection of the
    detected planes, in frames per second."""
    import workloads
    N = int(proj.shape[1])
    from paper_2501_13664_amd._lib import lib
    ws = torch.empty(lib().drt3d_detect_planes_workspace_bytes(N, 0xFFF, 0), dtype=torch.uint8, device="cuda")
    found = {}

    def det():
        found["r"] = api.drt3d_detect_planes(proj, 0.05, 0.5, cap=1 << 16, workspace=ws)

    ms = _best_ms(torch, det, reps)
    nbytes = 4.0 * proj.numel()
    res = {"workload": "drt3d_detect_planes N=%d int32 (the forward's projections), cos_tol 0.05, threshold 0.5" % N,
           "ms": ms, "planes": found["r"][1], "output_GBps": nbytes / (ms / 1e3) / 1e9}
    Nr = 128
    vol, _ = workloads.room_scene(Nr)
    v = torch.from_numpy(vol).cuda()
    pr = torch.empty(api.drt3d_out_shape(Nr), dtype=torch.int32, device="cuda")
    fws = torch.empty(lib().drt3d_workspace_bytes(Nr, 0xFFF, 0), dtype=torch.uint8, device="cuda")
    dws = torch.empty(lib().drt3d_detect_planes_workspace_bytes(Nr, 0xFFF, 0), dtype=torch.uint8, device="cuda")
    bws = torch.empty(lib().drt3d_backproject_bins_workspace_bytes(Nr, 0xFFF, 0), dtype=torch.uint8, device="cuda")
    back = torch.empty((Nr, Nr, Nr), dtype=torch.int32, device="cuda")

    def scene():
        api.drt3d_forward(v, out=pr, workspace=fws)
        b, n = api.drt3d_detect_planes(pr, 0.05, 0.5, cap=4096, workspace=dws)
        api.drt3d_backproject_bins(b, Nr, out=back, workspace=bws)
        found["scene"] = n

    sms = _best_ms(torch, scene, reps + 2)
    marked = int(((back > 0) & (v > 0)).sum())
    res["room_scene"] = {"workload": "room scene N=128 (seed 11): forward + detection + backprojection",
                         "ms": sms, "frames_per_s": 1e3 / sms, "planes": found["scene"],
                         "occupied_voxels_on_detected_planes": marked / int(v.sum())}
    return res


def inverse_rate(api, torch, N=128, cycles=10, reps=2):
    """The iterative inverse (Sec. 5.2) of the 12-dodecant float32 DRT of the
    corners-and-centre cube (value 1 on the 8 corners and the centre voxel) at
    N = 128: `cycles` V-cycles, after the one-time eigenvalue setup."""
    import workloads
    f = torch.from_numpy(workloads.corners_and_centre(N).astype("float32")).cuda()
    b = api.drt3d_forward(f)
    from paper_2501_13664_amd._lib import lib
    ws = torch.empty(lib().drt3d_inverse_workspace_bytes(N), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lams = api.drt3d_inverse_lambdas(N, workspace=ws)
    setup_ms = (time.perf_counter() - t0) * 1e3
    out = torch.empty((N, N, N), dtype=torch.float32, device="cuda")
    errs = {}
    for c in (1, 2, 4, 6):
        api.drt3d_inverse(b, c, lams=lams, out=out, workspace=ws)
        errs[c] = float(torch.linalg.vector_norm(out - f) / torch.linalg.vector_norm(f))
    # timed without the profiler (its events around every launch cost time),
    # then one profiled call for the per-kernel split
    ms = _best_ms(torch, lambda: api.drt3d_inverse(b, cycles, lams=lams, out=out, workspace=ws), reps)
    errs[cycles] = float(torch.linalg.vector_norm(out - f) / torch.linalg.vector_norm(f))
    with api.profile() as prof:
        api.drt3d_inverse(b, cycles, lams=lams, out=out, workspace=ws)
        torch.cuda.synchronize()
    recs = prof.records
    calls = 1
    pass_ms = sum(v[0] for v in recs.values()) / calls
    return {"workload": "drt3d_inverse N=%d float32, 12 dodecants, corners-and-centre cube, %d V-cycles" % (N, cycles),
            "ms": ms, "ms_per_cycle": ms / cycles, "setup_ms": setup_ms, "eigenvalues": lams,
            "relative_error_after_cycles": errs,
            "transform_share": pass_ms / ms,
            "kernels": {k: {"ms_per_call": v[0] / calls, "launches_per_call": v[1] / calls} for k, v in recs.items()}}


def copy_calibration(torch):
    """Plain 1 GiB device copy, five times: the reference for the byte counters."""
    n = 1 << 28
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                      "launches": 5}), flush=True)


def stream_ceiling(api, torch, read_bytes, write_bytes, src, dst, reps=5):
    """The reference stream (drt3d_stream_probe) with a kernel's algorithmic
    read and write bytes: GB/s of the median of `reps` timed runs, the ceiling
    HBM allows for that mix of reads and writes."""
    read_bytes = int(read_bytes) // 16 * 16
    write_bytes = int(write_bytes) // 16 * 16
    api.stream_probe(src, read_bytes, dst, write_bytes)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        api.stream_probe(src, read_bytes, dst, write_bytes)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = sorted(times)[len(times) // 2]
    return {"GBps": (read_bytes + write_bytes) / (ms / 1e3) / 1e9, "ms": ms,
            "read_GB": read_bytes / 1e9, "write_GB": write_bytes / 1e9}


def attach_ceiling(roof, ceil):
    """Adds the same-mix stream ceiling to a roofline record."""
    roof["ceiling"] = {"GBps": ceil["GBps"], "frac_of_ceiling": roof["achieved"] / ceil["GBps"],
                       "reference": "drt3d_stream_probe moving the kernel's algorithmic bytes "
                                    "(%.2f GB read, %.2f GB written) in %.3f ms"
                                    % (ceil["read_GB"], ceil["write_GB"], ceil["ms"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-diff", action="store_true")
    ap.add_argument("--no-djt", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-inverse", action="store_true")
    ap.add_argument("--no-planes", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
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
        "compulsory_floor": floor_record(N, ms),
        "kernels": kernels,
    }
    if not args.no_adjoint:
        line["adjoint"] = adjoint_rate(api, torch, out, N)
        line["merge_net"] = merge_net_rate(api, torch, out)
        line["narrow_u8"] = narrow_rate(api, torch, vol_np, out)
    if not args.no_planes:
        line["plane_detection"] = planes_rate(api, torch, out)
    # the same-mix ceilings (they overwrite out and ws, which are done)
    out_bytes = 12 * 4 * N * N * (3 * N - 2)
    fwd_last = recs[dom][2] / recs[dom][1]
    attach_ceiling(line["roofline"], stream_ceiling(api, torch, fwd_last - out_bytes, out_bytes, ws, out))
    if "adjoint" in line:
        adj = line["adjoint"]
        attach_ceiling(adj["roofline"],
                       stream_ceiling(api, torch, out_bytes, adj["roofline"]["bytes_per_launch"] - out_bytes, out, ws))
    del ws
    torch.cuda.empty_cache()
    float_checks = []
    if not args.no_batched:
        line["batched_vs_per_volume"], chk = batched_speedup(api, torch)
        float_checks += chk
        torch.cuda.empty_cache()
    if not args.no_diff:
        line["differentiable_vs_per_volume"], chk = differentiable_speedup(api, torch)
        float_checks += chk
        torch.cuda.empty_cache()
    if not args.no_djt:
        line["djt"] = djt_rate(api, torch)
        torch.cuda.empty_cache()
    if not args.no_inverse:
        line["inverse"] = inverse_rate(api, torch)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(vol_np, float_checks)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
