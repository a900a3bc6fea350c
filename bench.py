#!/usr/bin/env python3
"""Throughput of the matrix-free immersed-boundary step on one MI355X.

Workload: the 128^3 Holzapfel-Ogden truncated-ellipsoid shell (127,008 nodes,
107,520 trilinear hexes, 17,920 endocardial pressure quads), dt = 5e-4,
p(t) = sin^2(pi t / T) with T = 100 dt, FP64, synthetic inputs from
paper_2503_22695_amd.inputs.  One step = FE force + pressure load, explicit
convection right-hand side, spreading, the Helmholtz and Poisson multigrid
solves (rtol 1e-10), projection, interpolation and position update, all in
libhipib's HIP kernels.

Prints one JSON line.  `value` is steps/s over the timed steps with every input
already resident in HBM.  `roofline` is for the dominant kernel class (the one
with the most time per step), and `roofline.other_kernels` gives the others:
each class is timed with HIP start/stop events that each dispatch stamps
itself (hipExtLaunchKernel), on the stream it runs on, during separate passes
of --roofline-steps steps after the timed region (events between launches
would slow the timed region itself); achieved = algorithmic bytes (or flops)
per launch / mean launch time.  `roofline_192` repeats the grid and coupling
kernels on the 192^3 shell with leaflets, whose solver arrays no longer fit
the last-level cache.  `cpu_baseline` is the FP64 CPU oracle timed on this
host on a bounded sample of the same workload (all threads, and one thread);
the oracle's run of the whole 100 steps also gives `parity_vs_oracle`, the
errors of the timed FP64 and mixed-precision runs.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FE_FLOP_PER_HEX = 3.7e3     # FE force, 2x2x2 Gauss points (algorithmic count)
METRIC = "IB steps/s at 128^3 HO shell: FP64 vs mixed-prec (err≤1e-6); adjoint/fwd time"


def cpu_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def host_cpu():
    """Model name and physical core count of this host (lscpu fields)."""
    model, cores, sockets = "unknown", None, None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            k, v = k.strip(), v.strip()
            if k == "Model name":
                model = v
            elif k == "Core(s) per socket":
                cores = int(v)
            elif k == "Socket(s)":
                sockets = int(v)
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    phys = cores * sockets if cores and sockets else None
    return model, phys


ORACLE_ONE_THREAD = r"""
import os, sys, time
sys.path.insert(0, {root!r})
import numpy as np
import oracle
from paper_2503_22695_amd import inputs
prob = inputs.workload("ho_shell_128")
fl = oracle.fluid_from_problem(prob)
mesh = oracle.MeshBuffers.from_problem(prob)
u, p, X = prob.initial_velocity(), np.zeros((prob.n,) * 3), prob.X0.copy()
u, p, X, _ = oracle.advance(fl, mesh, u, p, X, 0.0, 1, prob.p0, prob.T)
t = time.perf_counter()
u, p, X, _ = oracle.advance(fl, mesh, u, p, X, 0.0, {steps}, prob.p0, prob.T, first_step=1)
print(time.perf_counter() - t)
"""


def oracle_one_thread(steps: int):
    """s/step of the oracle on one thread (a child process with OMP_NUM_THREADS=1):
    1 warm-up step, then `steps` timed steps of the 128^3 shell."""
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", ORACLE_ONE_THREAD.format(root=ROOT, steps=steps)],
                         capture_output=True, text=True, env=env, timeout=600, check=True)
    return float(out.stdout.strip().splitlines()[-1]) / steps


def cpu_baseline_and_parity(prob, sample_steps: int, one_thread_steps: int, runs):
    """The CPU oracle as it stands: its run of the whole workload from t = 0 in
    pieces, the first `sample_steps` of which are timed (the baseline sample),
    then the errors of the GPU runs (state after the same steps) against it."""
    import numpy as np
    import oracle
    fl = oracle.fluid_from_problem(prob)
    mesh = oracle.MeshBuffers.from_problem(prob)
    u, p, X = prob.initial_velocity(), np.zeros((prob.n,) * 3), prob.X0.copy()
    t0 = time.perf_counter()
    u, p, X, _ = oracle.advance(fl, mesh, u, p, X, 0.0, sample_steps, prob.p0, prob.T)
    el = time.perf_counter() - t0
    progress(f"oracle: {sample_steps} steps timed ({el:.1f} s)")
    done = sample_steps
    while done < prob.n_steps:
        m = min(25, prob.n_steps - done)
        u, p, X, _ = oracle.advance(fl, mesh, u, p, X, 0.0, m, prob.p0, prob.T, first_step=done)
        done += m
        progress(f"oracle: {done} of {prob.n_steps} steps for the parity check")
    model, phys = host_cpu()
    base = {"value": sample_steps / el, "unit": "steps/s", "cores": cpu_threads(), "kind": "oracle",
            "sample": f"first {sample_steps} steps of the 128^3 shell workload from t=0 ({el:.1f} s, FP64 C "
                      f"with OpenMP grid loops, {cpu_threads()} threads)",
            "cpu_model": model, "physical_cores": phys}
    if one_thread_steps > 0:
        s1 = oracle_one_thread(one_thread_steps)
        base["one_thread"] = {"value": 1.0 / s1, "unit": "steps/s", "cores": 1,
                              "sample": f"steps 2..{1 + one_thread_steps} of the same workload, one thread"}
        progress("oracle: one-thread sample done")

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    def rel_inf(a, b):
        return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    par = {}
    for name, (ug, pg, Xg) in runs.items():
        pm, prm = pg - pg.mean(), p - p.mean()
        e = {"e_u": rel(ug, u), "e_p": rel(pm, prm),
             "e_X": float(np.max(np.abs(Xg - X)) / np.max(np.abs(X - prob.X0))),
             "u_inf": rel_inf(ug, u), "p_inf": rel_inf(pm, prm), "dX_l2": rel(Xg - prob.X0, X - prob.X0)}
        par[name] = e
    par["definition"] = ("after the timed 100 steps from t = 0, against the FP64 oracle's run: e_u, e_p (mean-free) "
                         "relative l2; e_X = max|X - X_ref| / max|X_ref - X0|; u_inf, p_inf relative max norms; "
                         "dX_l2 relative l2 of X - X0")
    return base, par


def workload_leg(torch, hipib, inputs, name, steps, **over):
    """FP64 steps/s of another workload (or configuration: `over`) over its
    first `steps` steps from t = 0 (3 warm-up steps on a copy of the state
    first)."""
    prob = inputs.workload(name)
    sim = hipib.Simulation(prob, **over)
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
    out = {"value": round(steps / el, 3), "unit": "steps/s", "steps": steps,
           "ms_per_step": round(1e3 * el / steps, 4), "dtype": "f64",
           "mg_cycles_per_step": {"helmholtz_max_component": float(np.mean(cyc[:, :3].max(1))),
                                  "poisson": float(np.mean(cyc[:, 3]))}}
    return out, sim, prob


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


def kernel_classes(hipib):
    """(timer, kernel name, algorithmic measure) of the timed kernel classes."""
    H = hipib
    return [
        (H.TIMER_SMOOTH_FINE_POISSON, "k_gs<double,2>",
         "finest-level red or black Gauss-Seidel half-sweep of the Poisson solve, 12 B/cell"),
        (H.TIMER_SMOOTH_FINE_HELMHOLTZ, "k_gs<double,1,true>",
         "finest-level over-relaxed red or black half-sweep of the Helmholtz solves, 16 B/cell per component"),
        (H.TIMER_RESID_RESTRICT, "k_resid_restrict<double>", "finest-level red residual and restriction, 13 B/cell"),
        (H.TIMER_PROLONG, "k_gs_prolong<double,16>",
         "first post-smoothing half-sweep with the trilinear coarse-grid correction folded in, 13 B/cell"),
        (H.TIMER_LEVEL_DOWN, "k_level_down<double>", "first coarse level, down half, 17 B per cell of that level"),
        (H.TIMER_LEVEL_UP, "k_level_up<double>", "first coarse level, up half, 21 B per cell of that level"),
        (H.TIMER_SMALL_VCYCLE, "k_exact_fwd_xy / k_exact_z / k_exact_inv_xy <32,double>",
         "coarsest level (32^3) solved exactly, three plane-parallel passes, 16 B per 32^3 cell each"),
        (H.TIMER_RESID_NORM, "k_resid_norm<false>", "residual norm, 16 B/cell per component"),
        (H.TIMER_CG_DOTS, "k_gs_dot<double>",
         "last two post-smoothing half-sweeps of the preconditioner, with r.z and z.q, 16 B/cell"),
        (H.TIMER_CG_DIR, "k_cg_dir<double>", "p, q = A z + beta q and p.q, 40 B/cell"),
        (H.TIMER_CG_UPDATE, "k_cg_update",
         "alpha from the p.q partials, x, r updates, ||r||^2 and sum-x partials, 48 B/cell"),
        (H.TIMER_REDUCE, "k_finalize / k_cg_scalars", "single-workgroup reductions, 8 B per partial"),
        (H.TIMER_RHS, "k_rhs_build",
         "fluid right-hand side with convection, u^n packed as the Helmholtz guess, 72 B/cell"),
        (H.TIMER_DIVERGENCE, "k_divergence_packed",
         "Poisson right-hand side from the packed u*, with sum-b and sum-b^2 partials, 32 B/cell"),
        (H.TIMER_PROJECT, "k_project_packed",
         "velocity correction from the packed u* and p, u and p written in natural layout, 64 B/cell"),
        (H.TIMER_PACK, "k_pack / k_unpack", "layout conversions, 16 B/cell per component"),
        (H.TIMER_SPREAD, "k_spread_tiles<8,double>",
         "spreading: 52 B/node (X, F, order) + 16 B per touched grid value (f read and written)"),
        (H.TIMER_INTERP, "k_interp_tiles<8,double>",
         "interpolation and position update: 52 B/node (X read and written, order) + 8 B per touched grid value"),
        (H.TIMER_FE_FORCE, "k_fe_force<double,Hex8>", "element forces, 3.7 kflop per hex (FP64 ALU)"),
    ]


def stencil_footprint(X, n):
    """Distinct (lattice, grid point) pairs in the 4x4x4 delta-kernel stencils of
    the nodes at X on the n^3 grid (the support of phi(r - i) for r the node's
    lattice coordinate: lattice d has offset 0 along d and 1/2 along the
    others), counted on the host from the stencil definition."""
    import numpy as np
    total = 0
    s = np.arange(4)
    for d in range(3):
        off = np.array([0.0 if e == d else 0.5 for e in range(3)])
        base = np.floor(X * n - off).astype(np.int64) - 1            # first stencil index per axis
        ix = (base[:, 0:1] + s) % n
        iy = (base[:, 1:2] + s) % n
        iz = (base[:, 2:3] + s) % n
        flat = (ix[:, :, None, None] + n * (iy[:, None, :, None] + n * iz[:, None, None, :])).reshape(-1)
        total += np.unique(flat).size
    return total


def time_classes(torch, hipib, sim, prob, t_start, steps, classes):
    """Per-class launch times over `steps` steps continuing the run on copies of
    its state; (launches, total_ms, bytes_per_launch) per timer."""
    out = {}
    ctx = sim.ctx
    for tid, _, _ in classes:
        u, p, X = sim.u.clone(), sim.p.clone(), sim.X.clone()
        ctx.timer_enable(tid)
        ctx.advance(u, p, X, t_start, steps, prob.p0, prob.T)
        torch.cuda.synchronize()
        out[tid] = ctx.timer_read()
        ctx.timer_enable(hipib.TIMER_OFF)
        del u, p, X
    return out


def roofline_table(hipib, tim, classes, steps, nodes_bytes, fe_flops):
    """Achieved GB/s (or TFLOP/s) of every timed class; sorted by time per step."""
    rows = {}
    for tid, name, what in classes:
        launches, ms, bpl = tim.get(tid, (0, 0.0, 0.0))
        if launches == 0:
            continue
        avg_s = ms * 1e-3 / launches
        row = {"what": what, "launches_per_step": round(launches / steps, 2),
               "avg_launch_us": round(avg_s * 1e6, 3), "ms_per_step": round(ms / steps, 4)}
        if tid == hipib.TIMER_FE_FORCE:
            ach = fe_flops / avg_s / 1e12
            row.update({"bound": "fp64-alu", "flops_per_launch": fe_flops, "achieved": round(ach, 3),
                        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4)})
        else:
            if tid in nodes_bytes:
                bpl = nodes_bytes[tid]
            ach = bpl / avg_s / 1e9
            row.update({"bound": "hbm", "bytes_per_launch": round(bpl), "achieved": round(ach, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4)})
        rows[name] = row
    return dict(sorted(rows.items(), key=lambda kv: -kv[1]["ms_per_step"]))


KERNEL_SOURCE = os.path.join(ROOT, "paper_2503_22695_amd", "csrc", "mg.hip")


# kernel classes with a committed counter summary: profiles/<prefix>_<workload>_hbm_traffic.md
TRAFFIC_PROFILES = {"k_gs<double,2>": "k_gs_poisson_fine", "k_gs<double,1,true>": "k_gs_helmholtz_sor_fine"}


def measured_traffic(kernel_class: str, workload: str = "128"):
    """HBM bytes per launch of the kernel class `kernel_class` from its
    committed counter summary, or None when there is none for this workload or
    the kernel code has changed since it was taken."""
    prefix = TRAFFIC_PROFILES.get(kernel_class)
    if prefix is None:
        return None
    path = os.path.join(ROOT, "profiles", f"{prefix}_{workload}_hbm_traffic.md")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    vals = {}
    for ln in lines:
        if ln.startswith("- ") and ": " in ln:
            k, v = ln[2:].split(": ", 1)
            vals[k.strip("`")] = v.strip().strip("`")
    if vals.get("kernel_code_sha256") != kernel_code_sha256() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def kernel_code_sha256(path: str = None) -> str:
    """sha256 of the multigrid source without its // comments, trailing blanks
    and empty lines: the code the counters were taken on (comment edits do not
    change it)."""
    import hashlib
    import re
    lines = []
    for ln in open(path or KERNEL_SOURCE, encoding="utf-8").read().splitlines():
        ln = re.sub(r"//.*$", "", ln).rstrip()
        if ln:
            lines.append(ln)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


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
    ap.add_argument("--cpu-steps", type=int, default=25, help="oracle steps timed for the CPU baseline")
    ap.add_argument("--cpu-one-thread-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-192", action="store_true", help="skip the 192^3 shell+leaflets leg")
    ap.add_argument("--steps-192", type=int, default=20)
    ap.add_argument("--no-lv", action="store_true", help="skip the 128^3 left-ventricle-law leg")
    ap.add_argument("--no-det", action="store_true", help="skip the deterministic-mode leg")
    ap.add_argument("--no-tet", action="store_true", help="skip the 64^3 P2-tetrahedra leg")
    ap.add_argument("--no-walls", action="store_true",
                    help="skip the walled 64^3 shell leg and the walled adjoint ratio")
    ap.add_argument("--roofline-steps", type=int, default=20,
                    help="steps of each separate pass that times one kernel class")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (memory-counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this library runs on one GPU only (the step is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2503_22695_amd import hipib, inputs

    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        copy_calibration(torch, args.copy_calibration_mib)
    prob = inputs.ho_shell()
    classes = kernel_classes(hipib)

    def run(precision):
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
        if not (torch.isfinite(sim.u).all() and torch.isfinite(sim.X).all()):
            raise RuntimeError("non-finite state after the timed run")
        return sim, t1 - t0, cyc

    sim, elapsed, cyc = run(hipib.FP64)
    steps_per_s = args.steps / elapsed
    progress(f"FP64 {args.steps} steps in {elapsed:.3f} s")
    t_end = args.steps * prob.dt
    # per-class kernel times on the state after the timed region
    Xh = sim.X.cpu().numpy()
    fp = stencil_footprint(Xh, prob.n)
    nodes_bytes = {hipib.TIMER_SPREAD: 52.0 * prob.n_nodes + 16.0 * fp,
                   hipib.TIMER_INTERP: 52.0 * prob.n_nodes + 8.0 * fp}
    tim = time_classes(torch, hipib, sim, prob, t_end, args.roofline_steps, classes)
    table = roofline_table(hipib, tim, classes, args.roofline_steps, nodes_bytes, FE_FLOP_PER_HEX * prob.n_elems)
    progress("per-kernel roofline passes done")
    gpu_state = {"fp64": tuple(t.cpu().numpy() for t in (sim.u, sim.p, sim.X))}
    phase_sim = sim
    for name in table:
        if name in TRAFFIC_PROFILES:
            table[name]["traffic"] = measured_traffic(name)
    dom_name = next(iter(table))
    dom = table[dom_name]
    roofline = {k: dom[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    roofline["traffic"] = measured_traffic(dom_name) if dom["bound"] == "hbm" else None
    roofline.update({
        "kernel": f"{dom_name}: {dom['what']}",
        "bytes_per_launch": dom.get("bytes_per_launch"), "launches_per_step": dom["launches_per_step"],
        "avg_launch_us": dom["avg_launch_us"], "ms_per_step": dom["ms_per_step"],
        "timing": f"HIP start/stop events stamped by each dispatch (hipExtLaunchKernel) on its stream, during "
                  f"{args.roofline_steps} further steps per kernel class run after the timed region",
        "other_kernels": {k: v for k, v in table.items() if k != dom_name},
        "stencil_footprint_values": fp,
    })
    # phase times over the same number of steps (a separate pass: one wait per step)
    u, p, X = sim.u.clone(), sim.p.clone(), sim.X.clone()
    phase_sim.ctx.set_phase_timing(True)
    phase_sim.ctx.advance(u, p, X, t_end, args.roofline_steps, prob.p0, prob.T)
    st = phase_sim.ctx.get_stats(u, X)
    phase_sim.ctx.set_phase_timing(False)
    phases = {k: round(v / max(st["timed_steps"], 1), 4) for k, v in st["phase_ms"].items()}
    diagnostics = {"J_min": st["J_min"], "J_max": st["J_max"], "volume": st["volume"],
                   "volume_change": st["volume"] / phase_sim.ctx.get_stats(None, torch.tensor(
                       np.ascontiguousarray(prob.X_ref), dtype=torch.float64, device="cuda").contiguous())["volume"]
                   - 1.0,
                   "kinetic_energy": st["kinetic_energy"], "max_abs_div": st["max_abs_div"]}
    del u, p, X

    mixed = None
    if not args.no_mixed:
        msim, melapsed, mcyc = run(hipib.MIXED)
        gpu_state["mixed"] = tuple(t.cpu().numpy() for t in (msim.u, msim.p, msim.X))
        mixed = {
            "value": round(args.steps / melapsed, 3), "unit": "steps/s",
            "ms_per_step": round(1e3 * melapsed / args.steps, 4),
            "over_fp64": round(elapsed / melapsed, 3),
            "dtype": "f32 V-cycles, element stresses (displacement form), spread weights and interpolation; "
                     "f64 outer residual, CG vectors and updates",
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

    larger, roof192 = None, None
    if not args.no_192:
        larger, lsim, lprob = workload_leg(torch, hipib, inputs, "shell_leaflets_192", args.steps_192)
        sub = [c for c in classes if c[0] in (hipib.TIMER_SMOOTH_FINE_POISSON, hipib.TIMER_SMOOTH_FINE_HELMHOLTZ,
                                               hipib.TIMER_RESID_RESTRICT, hipib.TIMER_PROLONG,
                                               hipib.TIMER_CG_DIR, hipib.TIMER_CG_UPDATE, hipib.TIMER_RHS,
                                               hipib.TIMER_SPREAD, hipib.TIMER_INTERP, hipib.TIMER_FE_FORCE)]
        fp192 = stencil_footprint(lsim.X.cpu().numpy(), lprob.n)
        nb192 = {hipib.TIMER_SPREAD: 52.0 * lprob.n_nodes + 16.0 * fp192,
                 hipib.TIMER_INTERP: 52.0 * lprob.n_nodes + 8.0 * fp192}
        tim192 = time_classes(torch, hipib, lsim, lprob, args.steps_192 * lprob.dt, 5, sub)
        roof192 = {"workload": "shell_leaflets_192: 192^3 grid, 280,740 nodes, 243,712 hexes "
                               "(one solver field 56.6 MB: the solve's arrays exceed the 256 MB last-level cache)",
                   "kernels": roofline_table(hipib, tim192, sub, 5, nb192, FE_FLOP_PER_HEX * lprob.n_elems),
                   "stencil_footprint_values": fp192}
        if "k_gs<double,2>" in roof192["kernels"]:
            roof192["kernels"]["k_gs<double,2>"]["traffic"] = measured_traffic("k_gs<double,2>", "192")
        del lsim
        progress("192^3 leg done")

    lv = None
    if not args.no_lv:
        lv, _, _ = workload_leg(torch, hipib, inputs, "lv_shell_128", 100)
        lv["law"] = ("Holzapfel-Ogden with sheet and fibre-sheet terms + active fibre tension; "
                     "base ring tethered axially and circumferentially")
        progress("left-ventricle-law leg done")

    tet = None
    if not args.no_tet:
        tet, _, _ = workload_leg(torch, hipib, inputs, "tet10_block_64", 20)
        tet["elements"] = "P2 tetrahedra, 4-point rule"
        progress("P2-tetrahedra leg done")

    det = None
    if not args.no_det:
        det, _, _ = workload_leg(torch, hipib, inputs, "ho_shell_128", 20, deterministic=1)
        det["mode"] = ("deterministic: nodes sorted by cell, each work item summed in node order into "
                       "its own box, boxes added per grid value in a fixed order; bitwise reproducible; "
                       "first 20 steps of the headline workload")
        progress("deterministic-mode leg done")

    walled = None
    if not args.no_walls:
        walled, _, _ = workload_leg(torch, hipib, inputs, "walled_shell_64", 20)
        walled["boundary"] = "walled box, (2n)^3 mirror-image grid"
        progress("walled-box leg done")

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
                   "mg": "Poisson: CG with one V(2,2) cycle, coarsest level 32^3 solved exactly; Helmholtz: "
                         "red-black SOR (Young) at the stop level; rtol 1e-10",
                   "mg_cycles_per_step": {"helmholtz_max_component": float(np.mean(cyc[:, :3].max(1))),
                                          "poisson": float(np.mean(cyc[:, 3]))}},
        "roofline": roofline,
        "phase_ms_per_step": phases,
        "diagnostics_after_run": diagnostics,
        "mixed_precision": mixed,
        "adjoint_over_forward": adjoint,
        "shell_leaflets_192": larger,
        "roofline_192": roof192,
        "lv_shell_128": lv,
        "tet10_block_64": tet,
        "walled_shell_64": walled,
        "deterministic_128": det,
    }
    if not args.no_cpu_baseline:
        if args.steps != prob.n_steps:
            gpu_state = {}      # the parity check compares the whole 100-step run only
        base, par = cpu_baseline_and_parity(prob, args.cpu_steps, args.cpu_one_thread_steps, gpu_state)
        out["cpu_baseline"] = base
        if gpu_state:
            out["parity_vs_oracle"] = par
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
