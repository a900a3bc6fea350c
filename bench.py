#!/usr/bin/env python3
"""Throughput of the matrix-free immersed-boundary step on one MI355X.

Workload: the 128^3 Holzapfel-Ogden truncated-ellipsoid shell (127,008 nodes,
107,520 trilinear hexes, 17,920 endocardial pressure quads), dt = 5e-4,
p(t) = sin^2(pi t / T) with T = 100 dt, FP64, synthetic inputs from
paper_2503_22695_amd.inputs.  One step = FE force + pressure load, explicit
convection right-hand side, spreading, three Helmholtz and one Poisson
multigrid solve (V(2,2) to 1e-10), projection, interpolation and position
update, all in libhipib's HIP kernels.

Prints one JSON line.  `value` is steps/s over the timed steps with every input
already resident in HBM.  `roofline` is for the dominant kernel (the finest
level red/black Gauss-Seidel sweep of the Poisson solve), timed with a HIP
event pair around each of its launches, on the launch stream, during a second
pass of --roofline-steps steps (events between launches would slow the timed
region itself).  `cpu_baseline` is the FP64 CPU
oracle timed on this host on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "IB steps/s at 128^3 HO shell: FP64 vs mixed-prec (err≤1e-6); adjoint/fwd time"


def cpu_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(prob, seconds: float):
    """The CPU oracle as it stands, timed on consecutive steps of the same
    workload from its initial state until `seconds` have elapsed."""
    import numpy as np
    import oracle
    fl = oracle.fluid_from_problem(prob)
    mesh = oracle.MeshBuffers.from_problem(prob)
    u = prob.initial_velocity()
    p = np.zeros((prob.n,) * 3)
    X = prob.X0.copy()
    steps, t = 0, 0.0
    start = time.perf_counter()
    while steps < 1 or time.perf_counter() - start < seconds:
        u, p, X, _ = oracle.advance(fl, mesh, u, p, X, t, 1, prob.p0, prob.T)
        t += prob.dt
        steps += 1
    el = time.perf_counter() - start
    return {"value": steps / el, "unit": "steps/s", "cores": cpu_threads(), "kind": "oracle",
            "sample": f"first {steps} steps of the 128^3 shell workload from t=0 "
                      f"({el:.1f} s, FP64 C with OpenMP grid loops)"}


def workload_leg(torch, hipib, inputs, name, steps):
    """FP64 steps/s of another workload over its first `steps` steps from t = 0
    (3 warm-up steps on a copy of the state first)."""
    prob = inputs.workload(name)
    sim = hipib.Simulation(prob)
    u, p, X = sim.u.clone(), sim.p.clone(), sim.X.clone()
    sim.ctx.advance(u, p, X, 0.0, 3, prob.p0, prob.T)     # warm-up on a copy
    del u, p, X
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.ctx.advance(sim.u, sim.p, sim.X, 0.0, steps, prob.p0, prob.T)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    cyc, _ = sim.ctx.step_stats()
    import numpy as np
    return {"value": round(steps / el, 3), "unit": "steps/s", "steps": steps,
            "ms_per_step": round(1e3 * el / steps, 4), "dtype": "f64",
            "mg_cycles_per_step": {"helmholtz_max_component": float(np.mean(cyc[:, :3].max(1))),
                                   "poisson": float(np.mean(cyc[:, 3]))}}


def larger_workload(torch, hipib, inputs, steps):
    """The 192^3 shell with two neo-Hookean leaflets (280,740 nodes, 243,712
    hexes, random divergence-free initial flow), where the solver's working set
    no longer fits the last-level cache."""
    return workload_leg(torch, hipib, inputs, "shell_leaflets_192", steps)


def tet_workload(torch, hipib, inputs):
    """P2 tetrahedra with the modified standard reinforcing law at the
    benchmark's settings (64^3 grid, dt 1e-3, one face penalised): 6,000 tets,
    9,261 nodes (27,783 solid DoFs), its 20-step run."""
    out = workload_leg(torch, hipib, inputs, "tet10_block_64", 20)
    out["elements"] = "P2 tetrahedra, 4-point rule"
    return out


def walled_workload(torch, hipib, inputs):
    """The Holzapfel-Ogden shell in a walled 64^3 box (no slip, no penetration),
    solved on its 128^3 mirror-image grid: its first 20 steps."""
    out = workload_leg(torch, hipib, inputs, "walled_shell_64", 20)
    out["boundary"] = "walled box, (2n)^3 mirror-image grid"
    return out


def lv_workload(torch, hipib, inputs):
    """The 128^3 shell with the full Holzapfel-Ogden law (sheet and fibre-sheet
    terms), transmural sheets, the active-tension pulse and the base constraint
    (penalty tethers): its whole 100-step run."""
    out = workload_leg(torch, hipib, inputs, "lv_shell_128", 100)
    out["law"] = ("Holzapfel-Ogden with sheet and fibre-sheet terms + active fibre tension; "
                  "base ring tethered axially and circumferentially")
    return out


def adjoint_ratio(torch, hipib, inputs, name="ho_block_64",
                  label="ho_block_64: 64^3 grid, 12^3 HO hexes, 50 steps, checkpoints every 10, FP64"):
    """Adjoint workload: 64^3 grid, Holzapfel-Ogden block of 12^3 hexes, 50
    steps, loss |X^N - X_target|^2 with X_target from a run at perturbed
    parameters; (checkpointed forward + backward) time over plain forward time,
    FP64, checkpoints every 10 steps.  name selects the same block in a walled
    box."""
    prob = inputs.workload(name)
    dev = torch.device("cuda", 0)
    theta = torch.tensor(prob.materials[0].params[:4], dtype=torch.float64)
    X0 = torch.tensor(prob.X0, dtype=torch.float64, device=dev)
    ro = hipib.Rollout(prob, checkpoint_every=10)
    Xt = ro.forward(theta * torch.tensor([1.1, 0.9, 1.1, 0.9], dtype=torch.float64), X0,
                    keep_checkpoints=False).clone()

    def grad_pass():
        th = theta.clone().requires_grad_(True)
        X0r = X0.clone().requires_grad_(True)
        L = ((hipib.IBRollout().apply(th, X0r, ro) - Xt) ** 2).sum()
        L.backward()
        return th

    # warm-up: one plain forward and one gradient pass (the first backward pass
    # creates the rollout's second context and stream for the overlapped
    # recomputation, a one-time set-up)
    ro.forward(theta, X0, keep_checkpoints=False)
    grad_pass()
    fwds, boths = [], []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ro.forward(theta, X0, keep_checkpoints=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        th = grad_pass()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fwds.append(t1 - t0)
        boths.append(t2 - t1)
    fwd, both = sorted(fwds)[1], sorted(boths)[1]
    return {"ratio": round(both / fwd, 3), "definition": "(checkpointed forward + backward) / plain forward, "
                                                       "medians of 3 after a warm-up gradient pass",
            "backward_over_forward": round((both - fwd) / fwd, 3), "forward_ms": round(1e3 * fwd, 2),
            "forward_plus_backward_ms": round(1e3 * both, 2),
            "workload": label,
            "grad_theta": [float(v) for v in th.grad]}


KERNELS = {}  # timer id -> description, filled once the library is loaded
KERNEL_SOURCE = os.path.join(ROOT, "paper_2503_22695_amd", "csrc", "mg.hip")


def measured_traffic(kernel: str):
    """HBM bytes per launch of the roofline kernel (e.g. "k_level_down") from the
    committed counter summary profiles/<kernel>_poisson_fine_128_hbm_traffic.md,
    or None when the kernel source has changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_poisson_fine_128_hbm_traffic.md")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    vals = {}
    for ln in lines:
        if ln.startswith("- ") and ": " in ln:
            k, v = ln[2:].split(": ", 1)
            vals[k.strip("`")] = v.strip().strip("`")
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if vals.get("kernel_source_sha256") != src or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def copy_calibration(torch, mib: int):
    """A plain device-to-device copy of `mib` MiB, three times: the reference
    kernel for scaling the memory counters of a profiled run."""
    n = mib * 1024 * 1024 // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def progress(msg: str):
    """One line per finished leg on stderr (stdout carries the JSON line only)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-192", action="store_true", help="skip the 192^3 shell+leaflets leg")
    ap.add_argument("--steps-192", type=int, default=20)
    ap.add_argument("--no-lv", action="store_true", help="skip the 128^3 left-ventricle-law leg")
    ap.add_argument("--no-tet", action="store_true", help="skip the 64^3 P2-tetrahedra leg")
    ap.add_argument("--no-walls", action="store_true",
                    help="skip the walled 64^3 shell leg and the walled adjoint ratio")
    ap.add_argument("--roofline-steps", type=int, default=20,
                    help="steps of the separate pass that times the roofline kernel")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (memory-counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs one GPU only (the step is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2503_22695_amd import hipib, inputs

    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        copy_calibration(torch, args.copy_calibration_mib)
    prob = inputs.ho_shell()

    def run(precision, timer):
        sim = hipib.Simulation(prob, precision=precision)
        ctx = sim.ctx
        # warm-up on a copy of the initial state (also settles the predicted cycle counts)
        u, p, X = sim.u.clone(), sim.p.clone(), sim.X.clone()
        if args.warmup > 0:
            ctx.advance(u, p, X, 0.0, args.warmup, prob.p0, prob.T)
        torch.cuda.synchronize()
        del u, p, X
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.advance(sim.u, sim.p, sim.X, 0.0, args.steps, prob.p0, prob.T)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cyc, _ = ctx.step_stats()
        tim = {}
        if timer:
            # roofline passes: the next steps of the same run, on copies, with
            # dispatch-stamped events on every launch of one finest-level
            # Poisson kernel class per pass
            t_end = args.steps * prob.dt
            for kind in KERNELS:
                u, p, X = sim.u.clone(), sim.p.clone(), sim.X.clone()
                ctx.timer_enable(kind)
                ctx.advance(u, p, X, t_end, args.roofline_steps, prob.p0, prob.T)
                torch.cuda.synchronize()
                tim[kind] = ctx.timer_read()
                ctx.timer_enable(hipib.TIMER_OFF)
                del u, p, X
        if not (torch.isfinite(sim.u).all() and torch.isfinite(sim.X).all()):
            raise RuntimeError("non-finite state after the timed run")
        return sim, t1 - t0, tim, cyc

    KERNELS.update({
        hipib.TIMER_SMOOTH_FINE_POISSON: "k_gs<double,2>: finest-level red or black Gauss-Seidel half-sweep "
                                         "of the Poisson solve (packed layout, 12 B/cell)",
    })
    sim, elapsed, tim, cyc = run(hipib.FP64, True)
    progress(f"FP64 {args.steps} steps in {elapsed:.3f} s and the roofline pass done")
    # the dominant kernel: the timed class with the most total time
    dom = max(tim, key=lambda k: tim[k][1])
    launches, kernel_ms, bytes_per_launch = tim[dom]
    steps_per_s = args.steps / elapsed

    mixed = None
    if not args.no_mixed:
        msim, melapsed, _, mcyc = run(hipib.MIXED, False)

        def rel(a, b):
            return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        dX = sim.X - torch.tensor(prob.X0, dtype=torch.float64, device=sim.X.device)
        mixed = {
            "value": round(args.steps / melapsed, 3), "unit": "steps/s",
            "ms_per_step": round(1e3 * melapsed / args.steps, 4),
            "dtype": "f32 V-cycles, element stresses (displacement form), spread weights and interpolation; f64 outer residual, CG vectors and updates",
            "error_vs_fp64_path": {
                "e_u": rel(msim.u, sim.u),
                "e_p": rel(msim.p - msim.p.mean(), sim.p - sim.p.mean()),
                "e_X": float((msim.X - sim.X).abs().max() / dX.abs().max()),
            },
            "mg_cycles_per_step": {"helmholtz_max_component": float(np.mean(mcyc[:, :3].max(1))),
                                   "poisson": float(np.mean(mcyc[:, 3]))},
        }
        del msim
        progress("mixed-precision leg done")

    adjoint = None
    if not args.no_adjoint:
        adjoint = adjoint_ratio(torch, hipib, inputs)
        progress("adjoint leg done")
        if not args.no_walls:
            adjoint["walled"] = adjoint_ratio(
                torch, hipib, inputs, "walled_ho_block_64",
                "walled_ho_block_64: the same block in a walled 64^3 box (128^3 image grid), "
                "50 steps, checkpoints every 10, FP64")
            progress("walled adjoint leg done")

    larger = None
    if not args.no_192:
        larger = larger_workload(torch, hipib, inputs, args.steps_192)
        progress("192^3 leg done")

    lv = None
    if not args.no_lv:
        lv = lv_workload(torch, hipib, inputs)
        progress("left-ventricle-law leg done")

    tet = None
    if not args.no_tet:
        tet = tet_workload(torch, hipib, inputs)
        progress("P2-tetrahedra leg done")

    walled = None
    if not args.no_walls:
        walled = walled_workload(torch, hipib, inputs)
        progress("walled-box leg done")

    avg_s = kernel_ms * 1e-3 / max(launches, 1)
    achieved = bytes_per_launch / avg_s / 1e9 if launches else 0.0
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(KERNELS[dom].split("<")[0]),
        "kernel": KERNELS[dom],
        "bytes_per_launch": bytes_per_launch, "launches": launches,
        "avg_launch_us": round(avg_s * 1e6, 3),
        "timing": f"HIP start/stop events stamped by each dispatch (hipExtLaunchKernel) on the library's stream, during {args.roofline_steps} "
                  "further steps run after the timed region",
        "other_kernels": {KERNELS[k].split(":")[0]: {"launches": v[0], "avg_launch_us": round(1e3 * v[1] / v[0], 3),
                                                     "achieved_GBs": round(v[2] * v[0] / (v[1] * 1e-3) / 1e9, 1)}
                          for k, v in tim.items() if k != dom and v[0] > 0},
    }
    out = {
        "metric": METRIC,
        "value": round(steps_per_s, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ho_shell_128", "grid": prob.n, "nodes": prob.n_nodes,
                   "hexes": prob.n_elems, "pressure_quads": prob.n_faces, "dt": prob.dt,
                   "mg": "V(2,2) red-black GS, rtol 1e-10",
                   "mg_cycles_per_step": {"helmholtz_max_component": float(np.mean(cyc[:, :3].max(1))),
                                          "poisson": float(np.mean(cyc[:, 3]))}},
        "roofline": roofline,
        "mixed_precision": mixed,
        "adjoint_over_forward": adjoint,
        "shell_leaflets_192": larger,
        "lv_shell_128": lv,
        "tet10_block_64": tet,
        "walled_shell_64": walled,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
