"""Throughput benchmark of the RLB-MIE-FD Allen-Cahn step on one MI355X.

Workload (default): 3D periodic, 512^3 nodes on (0,1)^3, eps = 0.02,
dt = 5e-4 (kappa = 0.0524288), a tanh sphere of radius 0.3 plus
Uniform[-0.01, 0.01] noise clipped to [-1, 1], energy and max-norm fused
every 100 steps.  One bench step is one time step of the scheme over the
whole field; the field is resident in HBM before timing starts.  --workload
2d / 1d time the 2D Neumann 1024^2 or the 1D periodic 256 workload instead.

Prints one JSON line: updates/s, the HBM roofline of the step kernel (16
algorithmic bytes per node update: read phi^n, write phi^{n+1}), the CPU
oracle timed on a bounded sample, the explicit comparison scheme, the other
two single-field workloads, and the adjoint cost ratio / batched speed-up.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12            # MI355X HBM3E, bytes/s
BYTES_PER_UPDATE = 16.0      # read phi^n + write phi^{n+1}
CSRC = os.path.join(ROOT, "paper_2312_07010_amd", "csrc")
KERNEL_SRC = {"k_march3d": "ace_march.hip", "k_tblock3d": "ace_tblock.hip",
              "k_tblock2d": "ace_tblock2d.hip", "k_tb3": "ace_tb3.h"}


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def committed_counters(kname, plane_chunk, region=None):
    """(figures for this launch shape, VALU peak) from the committed rocprofv3
    summary of the kernel, if it was taken on the current source of the kernel
    and of the device header; else None.  The 3D kernels are keyed by plane
    chunk (and, for k_tb3, by depth, region rows and rows per thread)."""
    path = os.path.join(ROOT, "profiles", f"{kname}_p512_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
        src = _sha(os.path.join(CSRC, KERNEL_SRC[kname])) + _sha(os.path.join(CSRC, "ace_device.h"))
    except (OSError, ValueError, KeyError):
        return None
    if t.get("kernel_src_sha") != src:
        return None
    if kname == "k_tb3":
        key = "{}x{}x{}/{}".format(*region, plane_chunk)
    else:
        key = str(plane_chunk) if kname == "k_tblock3d" else "any"
    return t.get("by_plane_chunk", {}).get(key), t.get("valu_peak_lane_instr_per_s")


def measured_traffic(kname, plane_chunk, region=None):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE runs (scaled by a copy of known size), if they were
    taken on the current source of that kernel and of the device header and
    at the same launch shape (planes per workgroup, region); else None."""
    cc = committed_counters(kname, plane_chunk, region)
    return cc[0].get("bytes_per_launch") if cc and cc[0] else None


def cpu_baseline(w, phi0_full, min_seconds=10.0):
    """The oracle as it stands, on a bounded sample of the same workload: the
    full field for as many steps as fill about `min_seconds`, once on all
    host threads and once on one thread."""
    import oracle
    p = oracle.Problem(w.d, w.N, w.L, w.R, w.eps, w.dt, w.bc)
    n = float(np.prod(p.shape))

    def leg(threads):
        prev = oracle.set_threads(threads)
        used = oracle.set_threads(0)
        phi, t, steps, k = phi0_full, 0.0, 0, 1
        while t < min_seconds:
            t0 = time.perf_counter()
            phi, _, _ = p.run(phi, k)
            t += time.perf_counter() - t0
            steps += k
            k = max(1, int((min_seconds - t) / (t / steps)))
        oracle.set_threads(prev)
        return {"value": n * steps / t, "unit": "grid-pt updates/s", "cores": used,
                "kind": "oracle",
                "sample": f"{'x'.join(map(str, p.shape))} field, {steps} step(s) "
                          f"({n * steps:.3g} updates, {t:.1f} s)"}

    out = leg(0)
    out["one_thread"] = leg(1)
    return out


# Depth of the 2D blocked kernel for the adjoint workload.  On 512^2 with
# 32-step checkpoint segments, depths 1..12 give forward / backward (ms):
# 1: 5.41 / 8.67, 2: 3.12 / 5.54, 3: 2.46 / 4.14, 4: 2.02 / 3.44,
# 5: 1.79 / 3.17, 6: 2.09 / 3.36, 8: 1.74 / 3.10, 10: 2.02 / 4.05,
# 12: 2.08 / 4.63.  Depth 8 is the fastest for both halves: its 16 x 48 tiles
# make 352 workgroups (240 at depth 5, fewer than the 256 CUs) and it divides
# the segments evenly.  The forward-step autotuner cannot see the reverse
# sweep and picks 5 or 8 (1.79 vs 1.73 ms).
ADJOINT_DEPTH = 8


def adjoint_ratio(ace, torch):
    """Backward / forward wall time: 2D Neumann 512^2, 1000 steps, checkpoints
    every 32 (forward = ace_forward_ckpt, backward = ace_backward), with the 2D
    blocked kernel at ADJOINT_DEPTH steps per launch in the forward, the
    recompute and the reverse sweep."""
    from paper_2312_07010_amd import inputs
    w = inputs.WADJ
    s = ace.Solver(w.d, w.N, w.L, w.R, w.eps, w.dt, w.bc)
    s.use_torch_stream()
    s.set_kernel(ace.ACE_KERNEL_TBLOCK, ADJOINT_DEPTH)
    phi0 = torch.tensor(inputs.uniform_field(s.shape, w.lo, w.hi, w.seed), device="cuda")
    k, per = s.get_kernel()
    kernel = f"{kernel_name(ace, w.d, k)} ({per} step(s) per launch)"
    tgt = torch.tensor(inputs.uniform_field(s.shape, w.lo, w.hi, w.extra["target_seed"]),
                       device="cuda")
    s.forward_ckpt(phi0, w.steps, w.extra["ckpt_every"])  # warm-up, same sizes
    s.backward(torch.zeros_like(phi0))
    torch.cuda.synchronize()
    phiT = torch.empty_like(phi0)
    lam = torch.empty_like(phi0)
    torch.sub(phiT, tgt, out=lam)  # loads torch's kernel outside the timed regions
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.forward_ckpt(phi0, w.steps, w.extra["ckpt_every"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.get_phi(phiT)
    torch.sub(phiT, tgt, out=lam)  # dL/dphi_T of L = |phi_T - target|^2 / 2
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.backward(lam)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    s.close()
    return (t3 - t2) / (t1 - t0), (t1 - t0) * 1e3, (t3 - t2) * 1e3, kernel


def slab_share(ace, torch, w, full, interior=64, halo=3, iters=200):
    """One GPU's share of the 3D workload split into 8 slabs along axis 0:
    a 64 x 512 x 512 slab with `halo` planes on each side, stepped `halo`
    steps between exchanges (3: one launch of the three-step blocked kernel,
    or a two-step and a one-step launch), the halos refreshed after every
    exchange interval by device copies standing in for the exchange with the
    neighbouring GPUs.  Here each slab is its own neighbour (periodic along
    axis 0), so the interior evolves exactly as a 64-plane periodic domain
    (checked bit for bit in the tests)."""
    n = w.N[1]
    P = interior + 2 * halo
    dx = (w.R[1] - w.L[1]) / n
    s = ace.Solver(3, [P, n, n], [0.0] * 3, [P * dx, w.R[1], w.R[2]], w.eps, w.dt, w.bc)
    s.use_torch_stream()
    s.set_kernel(ace.ACE_KERNEL_TBLOCK)
    a = torch.empty(P * n * n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    s.bind_fields(a, b)
    z0 = w.N[0] // 2 - interior // 2  # the central slab of the benchmark field `full`
    s.set_phi0(full[z0 - halo:z0 + interior + halo])
    tune = json.loads(s.autotune(20))["choice"]  # launch shape for the slab (restores the field)
    kernel, per_launch = s.get_kernel()

    def launch():
        s.step(halo)
        cur = a if s.field_ptr() == a.data_ptr() else b
        v = cur.view(P, n, n)
        v[:halo].copy_(v[interior:interior + halo])
        v[halo + interior:].copy_(v[halo:2 * halo])

    for _ in range(10):
        launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        launch()
    e1.record()
    torch.cuda.synchronize()
    per = e0.elapsed_time(e1) / 1e3 / iters
    s.close()
    return {"value": interior * n * n * halo / per, "unit": "grid-pt updates/s per GPU",
            "shape": f"{interior}x{n}x{n} interior + {halo}+{halo} halo planes",
            "steps_per_exchange": halo, "us_per_exchange_interval": per * 1e6,
            "steps_per_launch": per_launch, "plane_chunk": tune["zchunk"],
            "note": "halos refreshed by device copies in place of the exchange over xGMI"}


def batched_speedup(ace, torch):
    """The 4096-instance workload (half 1D, half 2D, mixed eps and BCs), 500
    steps: one persistent launch (after the batch autotuner picks its LDS
    limit) vs the same library's ace_step(500) called per instance in a loop
    on one stream (step calls only in both timed regions)."""
    from paper_2312_07010_amd import inputs
    descs = inputs.batch_instances()
    insts = [(x.d, [x.N] * x.d, [0.0] * x.d, [1.0] * x.d, x.eps, x.dt, x.bc) for x in descs]
    b = ace.Batch(insts)
    b.use_torch_stream()
    phi0 = [inputs.batch_phi0(i, shp) for i, shp in enumerate(b.shapes)]
    b.set_all(phi0)
    tune = json.loads(b.autotune(50))
    b.set_all(phi0)
    b.step(500)  # graph capture and warm-up
    b.set_all(phi0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(500)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    updates = float(sum(b.totals)) * 500
    b.close()
    solvers = []
    for i, inst in enumerate(insts):
        s = ace.Solver(*inst)
        s.use_torch_stream()
        s.set_phi0(phi0[i])
        solvers.append(s)
    for s in solvers[:8]:
        s.step(2)
    for i, s in enumerate(solvers):
        s.set_phi0(phi0[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(500)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    for s in solvers:
        s.close()
    return {"speedup": t_loop / t_batch, "batched_s": t_batch, "looped_s": t_loop,
            "batched_updates_per_s": updates / t_batch,
            "algorithmic_hbm_frac": BYTES_PER_UPDATE * updates / t_batch / HBM_PEAK,
            "resident_limit": tune["choice"]["resident_limit"], "depth": tune["choice"]["depth"],
            "region": tune["choice"]["region"]}


def batch_launch(ace, torch, steps=500, depth=4, resident_limit=8000, region=0):
    """The batched workload's persistent launches alone, at a fixed choice
    (region depth, LDS limit, region height: 0 for LDS-plane regions, 32 or
    64 for register-resident ones in a kernel of their own), issued directly
    (no graph) so that counter tools see them: one untimed and one timed
    call of `steps` steps."""
    from paper_2312_07010_amd import inputs
    descs = inputs.batch_instances()
    insts = [(x.d, [x.N] * x.d, [0.0] * x.d, [1.0] * x.d, x.eps, x.dt, x.bc) for x in descs]
    b = ace.Batch(insts)
    b.use_torch_stream()
    b.set_graphs(False)
    b.set_depth(depth)
    b.set_resident_limit(resident_limit)
    b.set_region(region)
    phi0 = [inputs.batch_phi0(i, shp) for i, shp in enumerate(b.shapes)]
    b.set_all(phi0)
    b.step(steps)
    b.set_all(phi0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    updates = float(sum(b.totals)) * steps
    b.close()
    return {"seconds": t, "updates_per_s": updates / t, "depth": depth, "resident_limit": resident_limit,
            "region": region}


WORKLOAD_DESC = {
    "3d": "3D Allen-Cahn RLB-MIE-FD step, periodic, 512^3 nodes on (0,1)^3, eps 0.02, dt 5e-4, "
          "tanh sphere r 0.3 + U[-0.01,0.01] noise, energy + max-norm fused every 100 steps",
    "2d": "2D Allen-Cahn RLB-MIE-FD step, homogeneous Neumann, 1024^2 stored nodes (N = 1022) on "
          "(0,1)^2, eps 0.01, dt 1e-3, U[-0.9,0.9], energy + max-norm fused every 100 steps",
    "1d": "1D Allen-Cahn RLB-MIE-FD step, periodic, 256 nodes on (-1,1), eps 0.02, dt 1e-3, "
          "U[-0.05,0.05], energy + max-norm fused every 100 steps",
}


def kernel_name(ace, d, kernel, region=None):
    if kernel == ace.ACE_KERNEL_TBLOCK:
        if d == 3 and region is not None and region[1] > 0:
            return "k_tb3"
        if d == 2 and region is not None and region[0] > 0:
            return "k_tb2"
        return "k_tblock3d" if d == 3 else "k_tblock2d"
    return {ace.ACE_KERNEL_MARCH: "k_march3d", ace.ACE_KERNEL_DIRECT: "k_step_direct",
            ace.ACE_KERNEL_RESIDENT: "k_resident"}.get(kernel, str(kernel))


def launches_in(steps, every, per_launch):
    """Step-kernel launches of ace_run_monitored(steps, every): each monitor
    interval starts a new launch."""
    n, left = 0, steps
    while left > 0:
        k = min(every, left)
        n += -(-k // per_launch)
        left -= k
    return n


def timed_workload(ace, torch, w, kernel="auto", plane_chunk=-1, autotune=True, steps=None,
                   warmup=100, every=100, keep=False, region3d=None, region2d=None):
    """ace_run_monitored(steps, every) on the workload's field, resident in
    HBM, after `warmup` untimed steps; timed by the host clock and by HIP
    events on the solver's stream (torch's current stream)."""
    from paper_2312_07010_amd import inputs
    steps = w.steps if steps is None else steps
    s = ace.Solver(w.d, w.N, w.L, w.R, w.eps, w.dt, w.bc)
    s.use_torch_stream()
    kid = {"auto": ace.ACE_KERNEL_AUTO, "march": ace.ACE_KERNEL_MARCH,
           "tblock": ace.ACE_KERNEL_TBLOCK, "direct": ace.ACE_KERNEL_DIRECT}[kernel]
    s.set_kernel(kid)
    coords = [s.coords(a) for a in range(w.d)]
    phi0 = inputs.initial_field(w, s.shape, coords)
    phi0_dev = torch.tensor(phi0, device="cuda")
    s.set_phi0(phi0_dev)
    tuning = None
    if region2d and w.d == 2:
        s.set_kernel(ace.ACE_KERNEL_TBLOCK, region2d[2])
        s.set_region2d(region2d[0], region2d[1])
    elif plane_chunk >= 0:
        s.set_plane_chunk(plane_chunk)
        if region3d:
            s.set_kernel(ace.ACE_KERNEL_TBLOCK)
            s.set_region3d(*region3d)
    elif kernel == "auto" and autotune:
        tuning = json.loads(s.autotune(20))
    k, per_launch = s.get_kernel()
    region = s.get_region3d() if w.d == 3 else (s.get_region2d() if w.d == 2 else None)
    s.set_phi0(phi0_dev)
    s.run_monitored(warmup, every)  # also loads every kernel variant used below
    torch.cuda.synchronize()
    s.set_phi0(phi0_dev)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    E, mx = s.run_monitored(steps, every)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ok = bool(np.all(np.diff(E) <= 1e-14 * np.abs(E[:-1])) and mx.max() <= 1 + 4 * 2.0 ** -53)
    if k == ace.ACE_KERNEL_RESIDENT:  # the whole monitored run is one launch
        per_launch, launches = steps, 1
    else:
        launches = launches_in(steps, every, per_launch)
    r = {"solver": s if keep else None, "phi0": phi0, "phi0_dev": phi0_dev if keep else None,
         "n": float(s.total), "steps": steps, "wall": wall, "gpu_ms": gpu_ms,
         "kernel": kernel_name(ace, w.d, k, region), "per_launch": per_launch, "region": region,
         "launches": launches, "plane_chunk": s.get_plane_chunk(),
         "tuning": tuning, "E": E, "mx": mx, "theorems_hold": ok}
    if not keep:
        s.close()
    return r


def timed_pop(ace, torch, w, steps=40, warmup=3):
    """The mesoscopic form (2d+1 populations per node) on the workload's
    field from equilibrium: `steps` steps of ace_pop_step, timed by the host
    clock and by HIP events on the handle's stream (torch's current one)."""
    from paper_2312_07010_amd import inputs
    g = ace.Pop(w.d, w.N, w.L, w.R, w.eps, w.dt, w.bc)
    g.use_torch_stream()
    s = ace.Solver(w.d, w.N, w.L, w.R, w.eps, w.dt, w.bc)
    coords = [s.coords(a) for a in range(w.d)]
    s.close()
    phi0 = torch.tensor(inputs.initial_field(w, g.shape, coords), device="cuda")
    g.set_phi0(phi0)
    g.step(warmup)
    g.set_phi0(phi0)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = e0.elapsed_time(e1) / 1e3
    q, n = g.q, float(g.total)
    # the carried form (the default for d >= 2) reads phi and writes the q
    # populations and phi: 8 q + 16 bytes per node update; reading and
    # writing all q populations (the fused form) would be 16 q
    per = 8.0 * q + 16.0
    out = {"value": n * steps / wall, "unit": "grid-pt updates/s", "steps": steps,
           "ms_per_step": wall * 1e3 / steps, "avg_launch_us": gpu_s / steps * 1e6,
           "kernel": "k_pop_update, carried phi (1 step per launch)",
           "populations": q, "bytes_per_update": per,
           "roofline_frac": per * n * steps / gpu_s / HBM_PEAK,
           "frac_at_16q_bytes": 16.0 * q * n * steps / gpu_s / HBM_PEAK,
           "device_bytes": g.device_bytes, "fd_device_bytes": int(2 * 8 * n)}
    g.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="3d", choices=["3d", "2d", "1d", "pop3d"],
                    help="the timed workload (default: the 3D 512^3 benchmark; pop3d: the same "
                         "field in the mesoscopic form, 7 populations per node)")
    ap.add_argument("--steps", type=int, default=0, help="timed steps (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the CPU baseline and the adjoint/batched/other-workload side metrics")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU-baseline sample length per leg (all threads, one thread)")
    ap.add_argument("--kernel", default="auto", choices=["auto", "march", "tblock", "direct"],
                    help="step kernel (auto = the library's choice)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the library's autotuner (kernel and plane-chunk choice)")
    ap.add_argument("--plane-chunk", type=int, default=-1, metavar="P",
                    help="fix the 3D blocked kernel's planes per workgroup, 0 = persistent grid "
                         "(skips the autotuner)")
    ap.add_argument("--region2d", default="", metavar="R,T,K",
                    help="2D workload without the autotuner: region rows R, rows per thread T (0,0: the "
                         "LDS-plane kernel) and depth K")
    ap.add_argument("--batch-region", type=int, default=0, choices=[0, 32, 64], metavar="ROWS",
                    help="batch-launch only: region height of the large 2D instances (0: LDS-plane regions)")
    ap.add_argument("--batch-depth", type=int, default=4, metavar="K",
                    help="batch-launch only: steps per region round")
    ap.add_argument("--region3d", default="", metavar="D,R,T",
                    help="with --plane-chunk: the 3D blocked kernel's depth D, region rows R and rows "
                         "per thread T (2,0,0: the two-step kernel)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="REPS",
                    help="only copy a 1 GiB device buffer REPS times (a plain copy kernel of "
                         "known size, for scaling HBM counters) and report its bandwidth")
    ap.add_argument("--only", choices=["adjoint", "batched", "batch-launch"], default=None,
                    help="run only the adjoint-ratio or the batched measurement (for profiling) "
                         "and print its result; batch-launch: only the batched workload's "
                         "persistent launch, issued without graph replay (for counter collection)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2312_07010_amd import ace, inputs
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)

    if args.calibrate_copy:
        n = 1 << 27  # 2^27 doubles = 1 GiB
        a = torch.rand(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.calibrate_copy):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.calibrate_copy
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n,
                          "avg_ms": ms, "GBps_read_plus_write": 16 * n / ms / 1e6}))
        return

    if args.only == "adjoint":
        ratio, fwd_ms, bwd_ms, adj_kernel = adjoint_ratio(ace, torch)
        print(json.dumps({"only": "adjoint", "adjoint_cost_ratio": ratio, "forward_ms": fwd_ms,
                          "backward_ms": bwd_ms, "kernel": adj_kernel}), flush=True)
        return
    if args.only == "batched":
        print(json.dumps(dict(only="batched", **batched_speedup(ace, torch))), flush=True)
        return
    if args.only == "batch-launch":
        print(json.dumps(dict(only="batch-launch", **batch_launch(ace, torch, depth=args.batch_depth,
                                                                      region=args.batch_region))), flush=True)
        return

    if args.workload == "pop3d":
        w = inputs.W3D
        steps = args.steps or 40
        r = timed_pop(ace, torch, w, steps, args.warmup if args.warmup < 20 else 3)
        print(json.dumps({
            "metric": "FP64 grid-pt updates/s + % HBM roofline; adjoint cost ratio; batched vs looped",
            "value": r["value"], "unit": "grid-pt updates/s", "n_gpus": 1, "steps": steps,
            "warmup": 3, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "mesoscopic form (7 populations per node) of " + WORKLOAD_DESC["3d"],
                       "nodes": int(np.prod(w.N)), "monitor_every": 0},
            "roofline": {"bound": "hbm", "achieved": r["roofline_frac"] * HBM_PEAK / 1e9,
                         "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": r["roofline_frac"],
                         "traffic": None, "kernel": r["kernel"],
                         "bytes_per_launch": r["bytes_per_update"] * np.prod(w.N),
                         "avg_launch_us": r["avg_launch_us"]},
            "population_rlb": r}), flush=True)
        return
    w = {"3d": inputs.W3D, "2d": inputs.W2D, "1d": inputs.W1D}[args.workload]
    steps = args.steps or w.steps
    print(f"[bench] {w.name}: {steps} steps", file=sys.stderr, flush=True)
    region3d = tuple(int(v) for v in args.region3d.split(",")) if args.region3d else None
    region2d = tuple(int(v) for v in args.region2d.split(",")) if args.region2d else None
    r = timed_workload(ace, torch, w, args.kernel, args.plane_chunk,
                       not args.no_autotune and region2d is None, steps, args.warmup, args.every, keep=True,
                       region3d=region3d, region2d=region2d)
    s = r["solver"]
    n = r["n"]
    value = n * steps / r["wall"]
    print(f"[bench] {steps} steps in {r['wall']:.3f} s wall, {r['gpu_ms']:.1f} ms on the stream; "
          f"{r['kernel']} x{r['per_launch']}; max-norm {r['mx'].max():.6f}, energy "
          f"{r['E'][0]:.6g} -> {r['E'][-1]:.6g}", file=sys.stderr, flush=True)
    if not r["theorems_hold"]:
        print("[bench] WARNING: maximum principle or energy decay violated", file=sys.stderr)

    # roofline of the step kernel: average launch time over the timed region
    # (the region holds the step launches plus one monitor reduction per
    # monitor interval, a few microseconds each)
    avg_launch_s = r["gpu_ms"] / 1e3 / r["launches"]
    bytes_per_launch = BYTES_PER_UPDATE * n * r["per_launch"]
    achieved = bytes_per_launch / avg_launch_s
    traffic = measured_traffic(r["kernel"], r["plane_chunk"], r["region"])
    roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "traffic": traffic,
            "kernel": f"{r['kernel']} ({r['per_launch']} step(s) per launch)",
            "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_launch_s * 1e6}
    if traffic:
        # the counter-measured HBM bytes per launch over the same launch time:
        # the bandwidth the kernel really draws (achieved/frac above count the
        # algorithmic 16 B per node update, which temporal blocking undercuts)
        roof["hbm_achieved_gbps"] = traffic / avg_launch_s / 1e9
        roof["hbm_frac"] = traffic / avg_launch_s / HBM_PEAK
    if w.d == 3:
        roof["plane_chunk"] = r["plane_chunk"]
        if r["region"] and r["region"][1] > 0:
            roof["region"] = {"depth": r["region"][0], "rows": r["region"][1], "cols": 64,
                              "rows_per_thread": r["region"][2]}
    if w.d == 2 and r["region"] and r["region"][0] > 0:
        roof["region"] = {"depth": r["per_launch"], "rows": r["region"][0], "cols": 64,
                          "rows_per_thread": r["region"][1]}
    cc = committed_counters(r["kernel"], r["plane_chunk"], r["region"])
    if cc and cc[0] and cc[1] and "sq_per_launch" in cc[0]:
        # VALU issue time of one launch (committed SQ_INSTS_VALU x 64 lanes at
        # the peak lane-instruction rate) over the launch time measured here
        roof["valu_frac"] = cc[0]["sq_per_launch"]["SQ_INSTS_VALU"] * 64 / cc[1] / avg_launch_s

    out = {
        "metric": "FP64 grid-pt updates/s + % HBM roofline; adjoint cost ratio; batched vs looped",
        "value": value,
        "unit": "grid-pt updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall"] * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_DESC[args.workload], "nodes": int(n),
                   "monitor_every": args.every},
        "roofline": roof,
    }
    if r["tuning"] is not None:
        out["autotune"] = r["tuning"]["choice"]
    if not args.no_extras and w.d == 3:
        # the explicit comparison scheme (Remark 2) on the same workload and kernel
        phi0_dev = r["phi0_dev"]
        s.set_scheme(ace.ACE_SCHEME_FEX)
        s.set_phi0(phi0_dev)
        s.step(100)
        s.set_phi0(phi0_dev)
        torch.cuda.synchronize()
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        f0.record()
        s.step(steps)
        f1.record()
        torch.cuda.synchronize()
        fwall = time.perf_counter() - t0
        favg = f0.elapsed_time(f1) / 1e3 / -(-steps // r["per_launch"])
        out["fex_scheme"] = {"value": n * steps / fwall, "unit": "grid-pt updates/s",
                             "roofline_frac": bytes_per_launch / favg / HBM_PEAK,
                             "kernel": roof["kernel"]}
        s.set_scheme(ace.ACE_SCHEME_RLB_MIE)
        # the standalone reductions over the same field: the energy / max-norm
        # monitor pass and the phase volume of the radius diagnostics (each
        # reads the field once, 8 B per node; synchronous calls, host clock)
        red = {}
        for name, fn in (("energy_monitor", s.energy), ("phase_volume", s.phase_volume)):
            fn()
            t0 = time.perf_counter()
            for _ in range(20):
                fn()
            t = (time.perf_counter() - t0) / 20
            red[name] = {"ms": t * 1e3, "hbm_frac": 8.0 * n / t / HBM_PEAK}
        out["reductions"] = red
    s.close()
    phi0 = r["phi0"]
    del r
    torch.cuda.empty_cache()

    if not args.no_extras:
        for name, ow in (("workload_2d", inputs.W2D), ("workload_1d", inputs.W1D)):
            if ow is w:
                continue
            try:
                o = timed_workload(ace, torch, ow, warmup=args.warmup, every=args.every)
                upd = o["n"] * o["steps"]
                out[name] = {"value": upd / o["wall"], "unit": "grid-pt updates/s",
                             "ms_per_step": o["wall"] * 1e3 / o["steps"], "steps": o["steps"],
                             "kernel": f"{o['kernel']} ({o['per_launch']} step(s) per launch)",
                             "algorithmic_hbm_frac": BYTES_PER_UPDATE * upd / (o["gpu_ms"] / 1e3)
                             / HBM_PEAK,
                             "theorems_hold": o["theorems_hold"]}
            except Exception as e:  # report, never hide
                out[name] = {"error": repr(e)}
        if w.d == 3:
            try:
                out["population_rlb"] = timed_pop(ace, torch, w)
                out["population_rlb"]["fd_over_pop_rate"] = value / out["population_rlb"]["value"]
            except Exception as e:  # report, never hide
                out["population_rlb"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        if w.d == 3:
            try:
                out["slab_share_8gpu"] = slab_share(ace, torch, w, phi0)
                out["slab_share_8gpu"]["vs_single_domain_rate"] = out["slab_share_8gpu"]["value"] / value
            except Exception as e:  # report, never hide
                out["slab_share_8gpu"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        try:
            ratio, fwd_ms, bwd_ms, adj_kernel = adjoint_ratio(ace, torch)
            out["adjoint_cost_ratio"] = ratio
            out["adjoint_ms"] = {"forward": fwd_ms, "backward": bwd_ms, "kernel": adj_kernel}
        except Exception as e:  # report, never hide
            out["adjoint_cost_ratio"] = None
            out["adjoint_error"] = repr(e)
        try:
            bs = batched_speedup(ace, torch)
            out["batched_speedup"] = bs["speedup"]
            out["batched"] = bs
        except Exception as e:
            out["batched_speedup"] = None
            out["batched_error"] = repr(e)
        out["cpu_baseline"] = cpu_baseline(w, phi0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
