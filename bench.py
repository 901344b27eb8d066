#!/usr/bin/env python
"""Benchmark of the batched PNCG-IPC load step on one MI355X.

Workload (default): 2048 environments, each a 20x16x4 mm gel meshed with
25x20x8 hexes (4,914 vertices, 24,000 tets) pressed by an end-on peg
(r = 4 mm, 2,048 triangles) at a seeded pose, 20 press steps to a seeded
depth. A "step" is one load step of every env: continuation, culling, every
PNCG iteration to tolerance and the marker output.

Timing: warmup runs ceil(W / K) untimed launches of the timed sequence itself
(load steps 1..K of the 20-step schedule from rest, so at least W load steps),
each followed by a reset of every env to rest; then load steps 1..K (K <= 20,
load step 1 from rest included) are timed in one persistent launch. Every
launch of the step kernel in a run therefore has the timed launch's shape, and
a profiler's per-kernel average equals the timed launch's duration.

Prints one JSON line: env-steps/s of the batched launch, the roofline of the
step kernel from HIP-event timings, the unbatched ("plain") solver on the
same GPU for a sample of envs, and the CPU oracle on a bounded sample.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
FP64_PEAK = 78.6e12        # FLOP/s, MI355X FP64 vector (256 CU x 4 SIMD x 16 lanes x FMA x 2.4 GHz)
FLOPS_PER_TET_ITER = 600   # element flops per tet per PNCG iteration (reference schedule)
BYTES_PER_VERT_ITER = 384  # 16 vector passes x 3 coords x 8 B per PNCG iteration


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="load steps timed, 1..20 of the press schedule, from rest")
    ap.add_argument("--warmup", type=int, default=2,
                    help="untimed load steps before the timed run: ceil(W/K) launches of the timed "
                         "sequence, envs reset to rest after each")
    ap.add_argument("--workload", choices=["peg_batch_5k", "peg_batch_5ku", "mixed_batch"], default="peg_batch_5k",
                    help="peg_batch_5k: uniform 2048 x 5k gels (headline); peg_batch_5ku: the same batch on the "
                         "unstructured (Delaunay) 5k gel; mixed_batch: 512 envs over three gel sizes and three "
                         "indenters")
    ap.add_argument("--envs", type=int, default=0, help="0: the workload's own count")
    ap.add_argument("--precision", choices=["f64", "mixed"], default="mixed")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--dynamic", action="store_true",
                    help="the implicit-Euler form (inertia with lumped masses; one time step per load step)")
    ap.add_argument("--dt", type=float, default=1.0 / 60.0, help="time step of the dynamic form (s)")
    ap.add_argument("--density", type=float, default=1.1e-9,
                    help="mass density of the dynamic form (t/mm^3; 1.1e-9 = 1,100 kg/m^3)")
    ap.add_argument("--plain-envs", type=int, default=4, help="envs timed one launch each (0: skip)")
    ap.add_argument("--launch", choices=["sequence", "per-step", "graph"], default="sequence",
                    help="sequence: the K timed load steps of every env in one launch; per-step: one launch per "
                         "load step; graph: one replay of a captured HIP graph (env ordering and step kernel) "
                         "per load step")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="oracle budget (0: skip)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--outer-radius", type=float, default=0.0,
                    help="coarse candidate list margin in multiples of dhat (0: the library default)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the adjoint instead: 64 envs of the 5k gel with friction, 20 load steps "
                         "recorded forward, then one t2r_backward_sequence launch (prints its own JSON line)")
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="block-shape / pair-capacity autotuner (setup, not timed); auto: on for the "
                         "uneven mixed_batch, off for the uniform batch (whose shape the automatic rule "
                         "picks: 256 threads when the envs outnumber the compute units)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration) and exit")
    return ap.parse_args()


KERNEL_SOURCES = ("t2r_internal.h", "t2r_kernels.hip", "t2r_math.h")


def source_hash() -> str:
    """Hash of the sources the device code is compiled from: a traffic profile
    stays valid while they are unchanged (host-only changes do not move it)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_28475_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def _cpu_model() -> str:
    """The CPU model as lscpu reports it (else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _nproc() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_worker(job):
    """One env of the workload, load step 1 from rest, through the oracle's PNCG
    reference (numpy FP64, BLAS threads 1) with the same continuation rule as the
    GPU path, until `seconds` have passed. Returns (iterations, seconds spent in
    solves that iterated)."""
    workload, env_id, seconds, tol = job
    from oracle.geometry import slerp_pose
    from oracle.pncg import pncg_solve
    from oracle.sim import build, continuation_increment
    env = workload.envs[env_id]
    gel, ind, prob = build(workload.meshes[env.mesh], workload.indenters[env.indenter], env)
    q0, q1 = env.poses[0], env.poses[1]
    x = gel.X.copy()
    prob.set_lag(x, q0)
    deadline = time.perf_counter() + seconds
    iters, spent, tau = 0, 0.0, 0.0
    while tau < 1.0 and time.perf_counter() < deadline:
        prob.set_pose(slerp_pose(q0, q1, tau))
        dtau = continuation_increment(prob, x, q0, q1, tau, prob.d_min(x))
        tau = min(1.0, tau + dtau)
        prob.set_pose(slerp_pose(q0, q1, tau))
        t0 = time.perf_counter()
        x, info = pncg_solve(prob, x, tol=tol, deadline=deadline)
        if info["iters"] > 0:  # solves out of contact converge at once
            iters += info["iters"]
            spent += time.perf_counter() - t0
    return iters, spent


def cpu_baseline_measure(args, workload):
    """Times the oracle's PNCG reference on the host's cores: one env per process
    (envs 0..P-1 of the workload, P = the usable cores, at most 16), each running
    load step 1 from rest for about args.cpu_seconds. Returns the per-iteration
    time of one process; the caller scales it by the GPU run's PNCG iterations
    per env-step (same algorithm and tolerance). Runs before the GPU is touched,
    so that the pool's processes fork from a process without a HIP context."""
    import multiprocessing as mp
    nproc = _nproc()
    cores = max(1, min(nproc, 16, len(workload.envs)))
    jobs = [(workload, i, args.cpu_seconds, args.tol) for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    iters = sum(r[0] for r in res)
    busy = sum(r[1] for r in res)
    return {"cores": cores, "iters": iters, "busy_s": busy, "wall_s": wall,
            "s_per_iter": busy / max(iters, 1), "cpu_model": _cpu_model(), "nproc": nproc}


def cpu_baseline(meas, iters_per_env_step, workload_name):
    """env-steps/s of the oracle on the measured cores: every process solves its
    own env, so the rate is cores / (seconds per iteration x iterations per env-step)."""
    per_step = meas["s_per_iter"] * iters_per_env_step
    return {"value": meas["cores"] / per_step, "unit": "env-steps/s", "cores": meas["cores"],
            "kind": "oracle",
            "cpu_model": meas["cpu_model"], "nproc": meas["nproc"],
            "sample": (f"{workload_name}: envs 0..{meas['cores'] - 1}, one per process (numpy FP64 PNCG "
                       f"reference, BLAS threads 1), load step 1 from rest for {meas['busy_s'] / meas['cores']:.0f} s "
                       f"each: {meas['iters']} PNCG iterations, {meas['s_per_iter']:.2f} s per iteration and "
                       f"process; extrapolated to whole env-steps with the GPU run's "
                       f"{iters_per_env_step:.0f} PNCG iterations per env-step (same algorithm and tolerance)")}


def adjoint_bench(args):
    """Adjoint grads/s on the calibration-gradient workload: envs of the 5k gel
    pressed by the peg (10 steps to 0.6 mm) and slid (10 steps, 0.5 mm) with
    friction. Per env the loss is sum |u_20 - u_target|^2 over the final-step
    markers, the target simulated at the env's hidden theta* plus N(0, 0.01 mm)
    noise; the gradient with respect to theta = (E, nu, mu_f, dt, dw) is taken
    at the perturbed theta_0 through all 20 steps and the friction lag between
    them (t2r_backward_sequence). Timed: the backward launch (HIP events); the
    recorded forward at theta_0 is reported beside it."""
    import numpy as np
    import torch
    from paper_2603_28475_amd import t2r
    from paper_2603_28475_amd.sim import Sim
    from scenes.configs import adjoint_peg_5k
    n = args.envs if args.envs > 0 else 64
    w = adjoint_peg_5k(n_envs=n)
    sim = Sim.from_workload(w, t2r.default_opts(tol=args.tol, precision=0, max_iters=50000))
    poses = np.ascontiguousarray(np.stack([e.poses for e in w.envs])[:, 1:].transpose(1, 0, 2))
    S = poses.shape[0]

    def theta_of(key):
        th = np.zeros((n, 9))
        for i, e in enumerate(w.envs):
            d = e.extra[key]
            th[i] = [d["E"], d["nu"], d["mu"], *d["dt"], *d["dw"]]
        return th

    def run(th, record):
        ids = list(range(n))
        sim.ctx.set_materials(ids, [(th[i, 0], th[i, 1], th[i, 2], *sim.mats[i][3:]) for i in range(n)])
        sim.ctx.set_pose_offsets(ids, th[:, 3:9])  # the rigid pose offset, applied by the library
        sim.ctx.reset_envs(ids)
        if record:
            sim.record(S)
        return sim.step_sequence(poses)

    rng = np.random.default_rng(5)
    m_star, st_star = run(theta_of("theta_star"), False)
    target = m_star[-1] + torch.as_tensor(0.01 * rng.standard_normal(tuple(m_star[-1].shape)), device=m_star.device)
    stream = torch.cuda.current_stream()
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record(stream)
    markers, status = run(theta_of("theta0"), True)
    f1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = f0.elapsed_time(f1)
    fwd_ok = bool(((status.cpu().numpy() & t2r.ENV_CONVERGED) != 0).all())
    fwd_iters = float(np.mean([x["iters"] for x in sim.stats()]))
    dL_du = torch.zeros_like(markers)
    dL_du[-1] = 2.0 * (markers[-1] - target)
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b0.record(stream)
    g = sim.backward_sequence(dL_du)
    b1.record(stream)
    torch.cuda.synchronize()
    bwd_ms = b0.elapsed_time(b1)
    st = sim.stats()
    cg = np.array([x["iters"] for x in st])
    ok = all(x["status"] & t2r.ENV_CONVERGED for x in st) and bool(torch.isfinite(g).all())
    line = {"metric": "adjoint grads/s", "value": n / (bwd_ms * 1e-3), "unit": "grads/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": w.name, "envs": n, "load_steps": S, "friction": True,
                       "grad": "dL/d(E, nu, mu_f, dt, dw) of sum |u_20 - u_target|^2 through all steps",
                       "forward_tol_mm": args.tol, "cg_rel_tol": 1e-10,
                       "cg_iters_per_env_mean": float(cg.mean()), "cg_iters_per_env_max": int(cg.max()),
                       "cg_iters_per_step_mean": float(cg.mean()) / S,
                       "forward_pncg_iters_per_env": fwd_iters, "forward_converged": fwd_ok,
                       "all_converged": ok, "block_size": sim.ctx.get_opts().block_size or "auto (512 at <= 256 envs)"},
            "backward_ms": bwd_ms, "forward_ms": fwd_ms,
            "grads_per_s_with_forward": n / ((bwd_ms + fwd_ms) * 1e-3),
            "grad_env0": [float(v) for v in g[0].cpu().numpy()]}
    print(json.dumps(line), flush=True)


SCHEDULE_STEPS = 20  # load steps of every workload's press schedule


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the batched step shards "
              "environments across GPUs with no exchange inside a step; see DESIGN.md.",
              file=sys.stderr)
        sys.exit(2)
    W, K = args.warmup, args.steps
    if not 1 <= K <= SCHEDULE_STEPS or W < 0:
        print(f"--steps must be in 1..{SCHEDULE_STEPS} (the load steps of the press schedule, timed from "
              f"rest) and --warmup >= 0; got --steps {K} --warmup {W}", file=sys.stderr)
        sys.exit(2)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    import numpy as np
    import torch

    if torch.cuda.device_count() < 1:  # counts devices without creating a HIP context
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.adjoint:
        return adjoint_bench(args)
    if args.copy_calibration:
        # a plain copy kernel of known size: 1 GiB read + 1 GiB written per launch
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8}))
        return

    from scenes.configs import mixed_batch, peg_batch_5k
    if args.envs <= 0:
        args.envs = 512 if args.workload == "mixed_batch" else 2048
    if args.workload == "mixed_batch":
        workload = mixed_batch(n_envs=args.envs, n_steps=SCHEDULE_STEPS, precision=args.precision)
    else:
        workload = peg_batch_5k(n_envs=args.envs, n_steps=SCHEDULE_STEPS, precision=args.precision,
                                mesh="5ku" if args.workload == "peg_batch_5ku" else "5k")

    # the CPU oracle runs first, in processes forked before this one creates a HIP context
    cpu_meas = None
    if args.cpu_seconds > 0:
        cpu_meas = cpu_baseline_measure(args, workload)
        log(args, f"cpu oracle: {cpu_meas['cores']} processes, {cpu_meas['iters']} iterations, "
                  f"{cpu_meas['s_per_iter']:.2f} s/iteration")

    from paper_2603_28475_amd import t2r
    from paper_2603_28475_amd.sim import Sim

    prec = 0 if args.precision == "f64" else 1
    opts = t2r.default_opts(tol=args.tol, precision=prec, block_size=args.block, dynamic=int(args.dynamic),
                            dt=args.dt, density=args.density, outer_radius=args.outer_radius)
    t_build = time.perf_counter()
    # graph replays need a stream of their own (capture is not allowed on the default one)
    sim_stream = torch.cuda.Stream(device="cuda:0") if args.launch == "graph" else None
    sim = Sim.from_workload(workload, opts, stream=sim_stream)
    poses = torch.as_tensor(np.stack([e.poses for e in workload.envs]), dtype=torch.float64,
                            device="cuda:0")
    log(args, f"built {args.envs} envs in {time.perf_counter() - t_build:.1f}s")
    stream = sim.stream
    nv_env = np.array([workload.meshes[e.mesh].n_verts for e in workload.envs], dtype=np.float64)
    nt_env = np.array([workload.meshes[e.mesh].n_tets for e in workload.envs], dtype=np.float64)
    all_envs = list(range(args.envs))

    def seq(a, b, envs=slice(None)):  # poses of load steps a..b-1 as (steps, n_env, 7)
        return poses[envs, a:b].transpose(0, 1).contiguous()

    def warmup(sm, envs):
        """ceil(W / K) untimed runs of the timed sequence (load steps 1..K from rest),
        every env back at rest after each."""
        for _ in range(-(-W // K)):
            if args.launch == "sequence":
                sm.step_sequence(seq(1, K + 1, envs))
            elif args.launch == "graph":
                for s in range(1, K + 1):  # the first call captures the graph
                    sm.graph_step(poses[envs, s])
            else:
                for s in range(1, K + 1):
                    sm.step(poses[envs, s].contiguous())
            sm.stream.synchronize()
            sm.ctx.reset_envs(list(range(sm.n_env)))
        torch.cuda.synchronize()

    tuned = None
    use_tuner = args.autotune == "on" or (args.autotune == "auto" and args.workload == "mixed_batch")
    if use_tuner and args.block == 0:
        # setup (not timed): trial the first load step with each block shape, state restored
        tuned = sim.autotune(seq(1, 2), target_steps=K if args.launch == "sequence" else 1)
        log(args, f"autotune: {tuned}")

    warmup(sim, slice(None))
    log(args, f"warmup: {-(-W // K)} launch(es) of load steps 1..{K}, envs back at rest")

    # output buffers exist before the timed region (no allocation or fill inside it)
    n_m = sum(sim.n_m)
    markers = torch.zeros((K, n_m, 3), dtype=torch.float64, device="cuda:0")
    status = torch.zeros((K, args.envs), dtype=torch.int32, device="cuda:0")
    pose_seq = seq(1, K + 1)
    torch.cuda.synchronize()
    iters = []          # per launch: PNCG iterations of every env
    launch_ms = []
    t0 = time.perf_counter()
    if args.launch == "sequence":
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        sim.ctx.step_sequence(K, pose_seq, None, markers, None, status)
        end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        launch_ms.append(start.elapsed_time(end))
        st = sim.stats()
        iters.append(np.array([x["iters"] for x in st], dtype=np.int64))
        log(args, f"load steps 1..{K} in one launch: {launch_ms[0]:.1f} ms, iters/env-step mean "
                  f"{iters[0].mean() / K:.0f}, env total max {iters[0].max()}")
    else:
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        per_step = [pose_seq[k] for k in range(K)]
        for k in range(K):
            starts[k].record(stream)
            if args.launch == "graph":
                sim.graph_step(per_step[k])  # replay: pose copy, env ordering, step kernel
                ends[k].record(stream)
                with torch.cuda.stream(stream):
                    markers[k].copy_(sim.markers)
                    status[k].copy_(sim.status)
            else:
                sim.ctx.step(per_step[k], None, markers[k], None, status[k])
                ends[k].record(stream)
            st = sim.stats()  # synchronises; needed for the per-launch iteration counts
            iters.append(np.array([x["iters"] for x in st], dtype=np.int64))
            log(args, f"step {k + 1}: {starts[k].elapsed_time(ends[k]):.1f} ms, iters/env mean "
                      f"{iters[-1].mean():.0f} max {iters[-1].max()}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        launch_ms = [starts[k].elapsed_time(ends[k]) for k in range(K)]
    status_ok = bool(((status.cpu().numpy() & t2r.ENV_CONVERGED) != 0).all())
    value = args.envs * K / wall
    # roofline of the step kernel: algorithmic vector bytes per launch / launch time
    bytes_per_launch = [float((it * nv_env).sum()) * BYTES_PER_VERT_ITER for it in iters]
    achieved = float(np.mean([b / (t * 1e-3) for b, t in zip(bytes_per_launch, launch_ms)]))
    # HBM bytes of the same launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled
    # by a 1 GiB copy), valid only for the kernel source and launch they were taken with
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"t2r_step_kernel_{workload.name}_traffic.json")
    if os.path.exists(tfile) and args.launch == "sequence" and not args.dynamic:
        with open(tfile) as fh:
            tr = json.load(fh)
        if (tr.get("source_hash") == source_hash() and tr.get("envs") == args.envs
                and tr.get("precision") == args.precision and tr.get("load_steps") == K):
            traffic = tr.get("bytes_per_launch")
    # FP64-vector view of the same launch: element flops per iteration under the
    # reference schedule (about 350 per tet for energy, gradient and diagonal,
    # 250 per tet for the curvature), against 78.6 TFLOP/s
    flops = float(sum((it * nt_env).sum() for it in iters)) * FLOPS_PER_TET_ITER
    alu_achieved = flops / (sum(launch_ms) * 1e-3)
    # time-based roofline (per env-iteration, each pass at its binding roof)
    t_roof_iter = (np.maximum(72 * nv_env / HBM_PEAK, 350 * nt_env / FP64_PEAK)
                   + np.maximum(48 * nv_env / HBM_PEAK, 250 * nt_env / FP64_PEAK) + 264 * nv_env / HBM_PEAK)
    t_roof = float(sum((it * t_roof_iter).sum() for it in iters))

    plain = None
    if args.plain_envs > 0:
        # unbatched: the same solver and launch mode, one env per context, on a sample of envs
        n = min(args.plain_envs, args.envs)
        sims = [Sim.from_workload(workload, opts, envs=[i],
                                  stream=torch.cuda.Stream(device="cuda:0") if args.launch == "graph" else None)
                for i in range(n)]
        for i_, sm in enumerate(sims):
            warmup(sm, slice(i_, i_ + 1))
        tp = time.perf_counter()
        for i_, sm in enumerate(sims):
            if args.launch == "sequence":
                sm.step_sequence(seq(1, K + 1, slice(i_, i_ + 1)))
            elif args.launch == "graph":
                for s in range(1, K + 1):
                    sm.graph_step(poses[i_:i_ + 1, s])
            else:
                for s in range(1, K + 1):
                    sm.step(poses[i_:i_ + 1, s].contiguous())
        torch.cuda.synchronize()
        dtp = time.perf_counter() - tp
        plain = {"value": n * K / dtp, "unit": "env-steps/s",
                 "sample": f"envs 0..{n - 1}, load steps 1..{K} from rest, one env per launch",
                 "batched_over_plain": value / (n * K / dtp)}

    iters_mean = float(sum(it.sum() for it in iters)) / (args.envs * K)
    # per-phase wall time of an env's workgroup per PNCG iteration (in-kernel clocks,
    # last launch), at the launch's occupancy
    st_last = sim.stats()
    it_tot = max(1, sum(x["iters"] for x in st_last))
    phase_names = ("outer_cull", "filter", "curv_elem", "curv_pairs", "ccd", "eval_elem", "eval_pairs",
                   "vector", "launch", "friction_lag")
    phase_us = {n: 1e3 * sum(x["phase_ms"][k] for x in st_last) / it_tot for k, n in enumerate(phase_names)}
    evals_per_iter = sum(x["evals"] for x in st_last) / it_tot
    lists_per_step = {k: sum(x[k] for x in st_last) / (args.envs * K) for k in ("outer_builds", "reculls")}
    cpu = cpu_baseline(cpu_meas, iters_mean, workload.name) if cpu_meas else None
    line = {
        "metric": "env-steps/s at fixed PNCG tol (batched)",
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * wall / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": workload.name, "envs": args.envs,
                   "gel_verts": sorted({int(m.n_verts) for m in workload.meshes.values()}),
                   "gel_tets": sorted({int(m.n_tets) for m in workload.meshes.values()}),
                   "indenters": sorted(workload.indenters),
                   "load_steps_timed": f"1..{K} of {SCHEDULE_STEPS}, from rest", "tol_mm": args.tol,
                   "precision": args.precision, "all_converged": bool(status_ok),
                   "form": (f"dynamic (dt {args.dt:g} s, density {args.density:g} t/mm^3)" if args.dynamic
                            else "quasi-static"),
                   "pncg_iters_per_env_step": iters_mean, "launch": args.launch,
                   "phase_us_per_env_iter": {k: round(v, 2) for k, v in phase_us.items()},
                   "eval_passes_per_iter": round(evals_per_iter, 3),
                   "outer_radius_dhat": args.outer_radius if args.outer_radius > 0 else 6.0,
                   "list_builds_per_env_step": {k: round(v, 3) for k, v in lists_per_step.items()},
                   "block_size": sim.ctx.get_opts().block_size or 256,
                   "autotune_trial_ms": tuned["trial_ms"] if tuned else None},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": traffic,
                     "kernel": "t2r_step_kernel", "launch_ms": launch_ms,
                     "alu": {"achieved": alu_achieved / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                             "frac": alu_achieved / FP64_PEAK},
                     "t_roof_frac": t_roof / (sum(launch_ms) * 1e-3)},
        "plain": plain,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
