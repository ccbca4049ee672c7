"""Benchmark of the implicit DG hot path on one MI355X.

Workload (default): flow past a cylinder on a curved O-grid annulus, r in
[0.5, 10], 32 radial x 64 angular x 8 spanwise hexahedra (span pi), P = 4
(5^3 modes, 6^3 Gauss points), quadratic isoparametric maps, no-slip wall and
far field, Re 3900, Ma 0.2, 5 conserved variables in FP64 (10.24 M
unknowns), SDIRK2 at CFL 20 on the smallest element, GMRES(30) with rtol
5e-2, BRJ(7), Newton tolerance 1e-8, preconditioner frozen for 10 steps (the
paper's settings).  The fluid starts at rest and the far field sets it
moving; the warm-up steps ramp dt from dt/100 up to dt.

A timed "step" is one implicit SDIRK step (every stage: Newton, GMRES,
Jacobian-free matvecs, BRJ sweeps); the timed region starts with a
preconditioner build, as the first step of each freeze window does.

Printed JSON line: value = DG residual DOFs/s of the residual evaluation
(per-variable DoF N_e (P+1)^d per evaluation, back-to-back evaluations with
the state resident in HBM), ms_per_step = implicit-step time; the dominant
kernel's roofline (the BRJ sweep), the residual's own roofline, the DOF/s
the timed steps deliver, the precision forms (FP64 / FP32 / BF16 blocks) on
this workload and on the 16^3 P = 3 Taylor-Green cube, the learned Newton
guess on the 2D Taylor-Green workload, and the CPU oracle baseline (the
explicit ERK2 comparison with --explicit).
"""
from __future__ import annotations

import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--P", type=int, default=None, help="polynomial order (default: the workload's; nq = P+2)")
    ap.add_argument("--pc", default=None, help="preconditioner storage f64|f32|bf16 (default: workload's)")
    ap.add_argument("--brj-sweeps", type=int, default=None, help="BRJ sweeps J (default: the workload's, 7)")
    ap.add_argument("--pc-freeze", type=int, default=None,
                    help="steps a built preconditioner is kept (default: the workload's, 10 as in the paper)")
    ap.add_argument("--pc-refresh-its", type=int, default=None,
                    help="GMRES count of a Newton step above which the next stage rebuilds the blocks "
                         "(default: the workload's; 0 = fixed freeze only)")
    ap.add_argument("--ortho", default=None, choices=["mgs", "cgs2"],
                    help="GMRES orthogonalisation (default: the workload's, modified Gram-Schmidt)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision forms (FP64 / FP32 / BF16 blocks from the same state, on this "
                         "workload and on the 16^3 P = 3 Taylor-Green cube: their sweep's roofline, speed-up "
                         "and state difference against FP64)")
    ap.add_argument("--form-steps", type=int, default=2, help="steps per precision form")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned Newton guess (trained and timed on the 2D Taylor-Green workload)")
    ap.add_argument("--learned-workload", type=int, default=1,
                    help="workload the learned guess is trained and timed on")
    ap.add_argument("--learned-train", type=int, default=40, help="plain steps recorded to train the MLP")
    ap.add_argument("--learned-epochs", type=int, default=150, help="Adam passes over the recorded stages")
    ap.add_argument("--learned-held", type=int, default=5, help="held-out steps timed with each guess")
    ap.add_argument("--batch", action="store_true",
                    help="also time the batch of 64 independent 2D problems, batched against one by one")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--mms", action="store_true",
                    help="also run the steady manufactured Poiseuille comparison: implicit SDIRK2 (CFL 500 -> 5000) "
                         "against ERK2 at its largest stable CFL, both to steady state, P = 2, 3, 4")
    ap.add_argument("--mms-n", type=int, default=8, help="elements per direction of the manufactured case")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--explicit", action="store_true",
                    help="also run the explicit ERK2 comparison (its largest stable CFL and its time to reach the "
                         "same physical time as the timed implicit steps; 2-3 minutes on the cylinder)")
    ap.add_argument("--kernel-reps", type=int, default=100,
                    help="back-to-back residual evaluations per timing repeat (median of 5 repeats)")
    ap.add_argument("--three-kernel", action="store_true",
                    help="--mode residual: evaluate with the three-kernel path instead of the fused kernel")
    ap.add_argument("--mode", default="full", choices=["full", "sweep", "copy", "residual"],
                    help="sweep: only build the preconditioner and apply it (for counter runs); "
                         "copy: a plain 1 GiB device copy (counter calibration); "
                         "residual: 20 residual evaluations (for kernel traces)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _oracle_residual_rate(disc, u0, dofs, budget_s):
    """Full oracle residual evaluations until budget_s has passed: (DOF/s,
    evaluations, wall s, threads used = CPU time / wall)."""
    disc.residual(u0)          # metrics and mass matrices outside the timed loop
    n = 0
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    while True:
        disc.residual(u0)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    return dofs * n / wall, n, wall, cpu / wall


def cpu_baseline(cfg, budget_s=12.0):
    """The CPU oracle on the host cores, as it stands: residual evaluations of
    the same workload (for the cylinder: every 256th element and its face
    neighbours) for about budget_s seconds with the BLAS thread pools limited
    to one thread and then left at their default (all host cores), and one
    full SDIRK2 step of the 2D Taylor-Green workload (8x8, P = 2, CFL 20,
    Newton alpha 1e-8) in both settings."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle.dg import make_disc, initial_state, restricted_disc
    from oracle.physics import Gas
    from oracle import solver as OS
    mesh = cfg.mesh()
    if cfg.geometry == "annulus":
        kinds, states = cfg.boundary()
        gas = Gas(gamma=cfg.gamma, Pr=cfg.Pr, Re=cfg.Re, Ma=cfg.Ma, visc_law=cfg.visc_law, T_ref_K=cfg.T_ref_K,
                  flux_mode=cfg.flux_mode, riemann=cfg.riemann)
        sample = list(range(0, mesh.n_elem, 256))
        disc, keep, _ = restricted_disc(gas, mesh.dim, cfg.P, cfg.nq, mesh.face_nbr, sample,
                                        geo_nodes=mesh.geo_nodes, geo_order=mesh.geo_order, bc_kind=kinds,
                                        bc_state=states)
        u0 = W.freestream_state(cfg, mesh.n_elem)[keep]
        dofs = len(keep) * (cfg.P + 1) ** cfg.dim
        what = (f"residual R(u) = M^-1 L(u) on {len(keep)} elements of the same workload: every 256th "
                f"element and its face neighbours (outer faces closed by far field), all counted")
    else:
        disc = make_disc(cfg, mesh)
        u0 = initial_state(disc, W.noise(disc.shape, cfg.seed), cfg.noise_amp)
        dofs = cfg.dofs()
        what = "full residual evaluations R(u) = M^-1 L(u) of the same workload (u = projected initial state)"
    res = {}
    for label, lim in (("one_thread", 1), ("all_cores", None)):
        with threadpool_limits(limits=lim):
            rate, n, wall, thr = _oracle_residual_rate(disc, u0, dofs, budget_s)
        res[label] = {"value": rate, "unit": "DOF/s", "cores": max(1, round(thr)), "threads_used": thr,
                      "sample": f"{n} x {what} in {wall:.1f} s wall"}
    # a full implicit step of the 2D Taylor-Green workload
    c1 = W.config(1)
    m1 = c1.mesh()
    d1 = make_disc(c1, m1)
    u1 = initial_state(d1, W.noise(d1.shape, c1.seed), c1.noise_amp)
    steps = {}
    for label, lim in (("one_thread", 1), ("all_cores", None)):
        with threadpool_limits(limits=lim):
            r0 = resource.getrusage(resource.RUSAGE_SELF)
            t0 = time.perf_counter()
            _, sto = OS.SDIRK(d1, OS.SolverOpts(scheme=c1.scheme)).step(u1, c1.dt())
            wall = time.perf_counter() - t0
            r1 = resource.getrusage(resource.RUSAGE_SELF)
        cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
        steps[label] = {"s_per_step": wall, "threads_used": cpu / wall,
                        "newton_its": [x.newton_its for x in sto]}
    allc = res["all_cores"]
    return {"value": allc["value"], "unit": "DOF/s", "cores": allc["cores"], "kind": "oracle",
            "sample": allc["sample"] + f"; BLAS pools at their default on a host of {os.cpu_count()} "
                                       f"logical CPUs",
            "one_thread": res["one_thread"],
            "oracle_step_tgv2d-8x8-p2": steps,
            "host_logical_cpus": os.cpu_count()}


def sweep_bytes(ctx, cfg, prec):
    """Algorithmic HBM bytes of one BRJ sweep launch averaged over the J
    sweeps of an apply: the stored block inverses once, the right-hand side
    in and the result out, and for the J-1 sweeps with an off-diagonal
    product the previous iterate and the face flux Jacobians."""
    E = ctx.n_elem
    nb = ctx.shape[1] * ctx.shape[2]
    n = ctx.n_unknowns
    sd = {"f64": 8, "f32": 4, "bf16": 2}[prec]
    sj = 8 if prec == "f64" else 4
    nqf = cfg.nq ** (cfg.dim - 1)
    J = cfg.brj_sweeps
    first = E * nb * nb * sd + 2 * n * 8
    other = first + n * 8 + E * 2 * cfg.dim * nqf * (cfg.dim + 2) ** 2 * sj
    extra = 0
    if cfg.geometry == "annulus":
        # curved elements: one mass-matrix product M q per apply (M read, q in, M q out)
        nm = (cfg.P + 1) ** cfg.dim
        extra = E * nm * nm * 8 + 2 * n * 8
    return (first + (J - 1) * other + extra) / J


def _source_hash(rel_path, marker=None):
    """sha256 (16 hex digits) of a source file, from `marker` to the end."""
    import hashlib
    text = open(os.path.join(ROOT, rel_path)).read()
    if marker is not None:
        if marker not in text:
            return None
        text = text[text.index(marker):]
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def _profile_record(name, tag):
    """The last `tag {json}` line of profiles/<name>, or None."""
    rec = None
    try:
        for line in open(os.path.join(ROOT, "profiles", name)):
            if line.startswith(tag + " "):
                rec = json.loads(line[len(tag) + 1:])
    except OSError:
        return None
    return rec


SWEEP_MARKER = "// ---------------------------------------------------------------- apply"
RESIDUAL_SOURCES = ("paper_2002_04222_amd/csrc/dgj_fused.h", "paper_2002_04222_amd/csrc/dgj_residual.h",
                    "paper_2002_04222_amd/csrc/dgj_physics.h", "paper_2002_04222_amd/csrc/dgj_kernels.h",
                    "paper_2002_04222_amd/csrc/dgj_tables.h")


def measured_traffic(prec, workload="tgv3d-16c-p3"):
    """HBM bytes per BRJ sweep launch from the committed counter runs of the
    workload, or None when the sweep's source (the apply section of its
    header, which holds the sweep kernel and its load helpers) has changed
    since they were taken."""
    try:
        rec = _profile_record(f"k_brj_sweep_{workload}_traffic.md", "TRAFFIC")
        h = _source_hash("paper_2002_04222_amd/csrc/dgj_precond.h", SWEEP_MARKER)
    except OSError:
        return None
    if rec is None or h is None or rec.get("sweep_section_sha256_16") != h:
        return None
    return rec.get(prec)


def residual_counters(workload):
    """Counted HBM bytes and FP64 operations of one residual evaluation from
    the committed counter runs, or None when the residual kernels' sources
    have changed since they were taken."""
    rec = _profile_record(f"residual_{workload}_counters.md", "COUNTERS")
    if rec is None:
        return None
    try:
        h = "".join(_source_hash(p) for p in RESIDUAL_SOURCES)
    except OSError:
        return None
    if rec.get("residual_sources_sha256_16") != h:
        return None
    return rec


FP64_PEAK_TFLOPS = 78.6


def residual_algorithmic(cfg, n_elem):
    """Algorithmic FP64 flops and compulsory HBM bytes of one residual
    evaluation (sum factorisation, each face flux once):
      per element and variable: the backward transform and its transpose,
        2 x 2 (Q n^d + Q^2 n^(d-1) + ... + Q^d n), and the collocation
        gradient and its transpose, 2 x 2 d Q^(d+1);
      per element: 250 flops per volume point (Euler and viscous fluxes),
        900 per face point of its d own faces (Riemann flux and the
        interior-penalty terms);
      curved elements add the metric products of the gradients and fluxes,
        2 x 2 d^2 (d+2) per volume point, and the dense inverse mass matrix,
        2 (d+2) n^(2d);
    bytes: the state in and R out (16 per unknown) and, on curved elements,
    the stored per-point metrics and inverse mass matrices."""
    d, n, Q = cfg.dim, cfg.P + 1, cfg.nq
    nv = d + 2
    tr = 2 * sum(Q ** k * n ** (d - k + 1) for k in range(1, d + 1))
    per_var = 2 * tr + 2 * (2 * d * Q ** (d + 1))
    per_elem = nv * per_var + 250 * Q ** d + 900 * d * Q ** (d - 1)
    nm, nq, nqf = n ** d, Q ** d, Q ** (d - 1)
    byts = 16.0 * n_elem * nv * nm
    if cfg.geometry == "annulus":
        per_elem += 4 * d * d * nv * nq + 2 * nv * nm * nm
        byts += 8.0 * n_elem * ((d * d + 1) * nq + 2 * d * (d * d + d + 1) * nqf + nm * nm)
    return per_elem * n_elem, byts


def residual_roofline(cfg, n_elem, res_ms):
    flops, byts = residual_algorithmic(cfg, n_elem)
    t = res_ms * 1e-3
    out = {"bound": "alu", "kernel": "k_res_fused",
           "achieved": flops / t / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": flops / t / 1e12 / FP64_PEAK_TFLOPS, "algorithmic_flops": flops,
           "compulsory_bytes": byts, "hbm_GBps_compulsory": byts / t / 1e9,
           "hbm_frac_compulsory": byts / t / 1e9 / HBM_PEAK_GBS, "avg_launch_ms": res_ms,
           "counted": None}
    rec = residual_counters(cfg.name)
    if rec is not None:
        out["counted"] = {k: rec[k] for k in ("traffic_bytes", "fp64_flops") if k in rec}
        if "traffic_bytes" in rec:
            out["counted"]["traffic_over_compulsory"] = rec["traffic_bytes"] / byts
        if "fp64_flops" in rec:
            out["counted"]["fp64_TFLOPs"] = rec["fp64_flops"] / t / 1e12
            out["counted"]["fp64_frac"] = rec["fp64_flops"] / t / 1e12 / FP64_PEAK_TFLOPS
    return out


def time_apply(ctx, q, o, stream, reps, J):
    """Median over 3 repeats of (reps back-to-back BRJ applies) / (reps J):
    the average sweep launch (plus, on curved meshes, 1/J of the apply's one
    mass-matrix product), with HIP events on the context's stream."""
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        ctx.precond_apply(q, o)
    times = []
    for _ in range(3):
        ev0.record(stream)
        for _ in range(reps):
            ctx.precond_apply(q, o)
        ev1.record(stream)
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1) / (reps * J))
    return sorted(times)[1]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 "
                                   "(sharding over several GPUs is designed, not built)"}))
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as W
    from paper_2002_04222_amd import Context

    cfg = W.config(args.workload)
    import dataclasses
    if args.P is not None:
        cfg = dataclasses.replace(cfg, P=args.P, nq=args.P + 2, name=cfg.name.rsplit("-p", 1)[0] + f"-p{args.P}")
    over = {"pc_precision": args.pc, "pc_freeze": args.pc_freeze, "brj_sweeps": args.brj_sweeps,
            "pc_refresh_its": args.pc_refresh_its, "ortho": args.ortho}
    cfg = dataclasses.replace(cfg, **{k: v for k, v in over.items() if v is not None and v != ""})
    mesh = cfg.mesh()
    dt = cfg.dt()
    curved = cfg.geometry == "annulus"
    log(f"workload {cfg.name}: {mesh.n_elem} elements, P={cfg.P}, dt={dt:.4f}, pc={cfg.pc_precision}")
    kinds, states = cfg.boundary()

    def make(prec, c=cfg, m=mesh):
        k, st = c.boundary()
        ctx = Context(m, c, pc_precision=prec, bc_kind=k, bc_state=st)
        u = ctx.empty()
        if c.geometry == "annulus":
            # fluid at rest plus seeded noise; the far field sets it moving
            u.copy_(torch.tensor(W.freestream_state(c, m.n_elem, at_rest=True), dtype=torch.float64,
                                 device="cuda"))
        else:
            noise = torch.tensor(W.noise(ctx.shape, c.seed), dtype=torch.float64, device="cuda")
            ctx.project_tgv(noise, c.noise_amp, u)
        return ctx, u

    if args.mode == "copy":
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copied 3 x 1 GiB")
        return
    t_setup = time.perf_counter()
    ctx, u = make(cfg.pc_precision)
    torch.cuda.synchronize()
    log(f"context created in {time.perf_counter() - t_setup:.1f} s")
    stream = torch.cuda.current_stream()
    if args.mode == "residual":
        R = ctx.empty()
        ctx.set_residual_kernels(not args.three_kernel)
        tuned, _ = ctx.autotune(u, reps=5)
        for _ in range(20):
            ctx.residual(u, R)
        torch.cuda.synchronize()
        log(f"20 residual evaluations ({'three kernels' if args.three_kernel else 'fused kernel'}, tile {tuned})")
        return
    if args.mode == "sweep":
        ctx.precond_build(u, dt * _lam(cfg.scheme))
        o = ctx.empty()
        for _ in range(3):
            ctx.precond_apply(u, o)
        torch.cuda.synchronize()
        log(f"3 BRJ applies ({3 * cfg.brj_sweeps} sweeps), {sweep_bytes(ctx, cfg, cfg.pc_precision):.4e} "
            f"algorithmic bytes per sweep")
        return

    # ---- residual throughput (the metric): inputs resident, back-to-back
    # launches; the fused kernel (the library's default), and for comparison
    # the three-kernel path with the per-point traces and face fluxes staged
    # in HBM; each with its workgroup sizes by the autotuner
    R = ctx.empty()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_residual():
        for _ in range(10):
            ctx.residual(u, R)
        times = []
        for _ in range(5):
            ev0.record(stream)
            for _ in range(args.kernel_reps):
                ctx.residual(u, R)
            ev1.record(stream)
            torch.cuda.synchronize()
            times.append(ev0.elapsed_time(ev1) / args.kernel_reps)
        return sorted(times)[2], min(times), max(times)

    ctx.set_residual_kernels(False)
    tuned3, _ = ctx.autotune(u, reps=10)
    res3_ms, _, _ = time_residual()
    log(f"three-kernel residual {res3_ms:.4f} ms (workgroups volume, face, lift {tuned3})")
    ctx.set_residual_kernels(True)
    tuned, tune_ms = ctx.autotune(u, reps=10)
    res_ms, tmin, tmax = time_residual()
    log(f"fused residual {res_ms:.4f} ms (median of 5 x {args.kernel_reps}; {tmin:.4f}-{tmax:.4f}; "
        f"workgroup {tuned[0]})")
    # Jacobian-free matvec (one residual at u + eps v): with eps fixed, as
    # the solver calls it inside GMRES (eps is set once per Newton
    # iteration), and with eps <= 0, where the library reduces ||u|| and
    # reads it back before each matvec
    dt_a = dt * _lam(cfg.scheme)
    Nu = ctx.empty()
    ctx.stage_residual(u, u, dt_a, Nu)
    v = torch.tensor(W.random_vector(mesh.n_elem, cfg.dim, cfg.P, seed=5), dtype=torch.float64, device="cuda")
    Jv = ctx.empty()
    eps_fixed = float(np.linalg.norm(u.cpu().numpy().ravel())) * 2.0 ** -26
    reps_mv = max(10, args.kernel_reps // 2)
    mv = {}
    for label, eps in (("fixed", eps_fixed), ("reduced", 0.0)):
        for _ in range(3):
            ctx.jfnk_matvec(u, Nu, u, dt_a, v, eps, Jv)
        ev0.record(stream)
        for _ in range(reps_mv):
            ctx.jfnk_matvec(u, Nu, u, dt_a, v, eps, Jv)
        ev1.record(stream)
        torch.cuda.synchronize()
        mv[label] = ev0.elapsed_time(ev1) / reps_mv
    mv_ms, mv_red_ms = mv["fixed"], mv["reduced"]
    del Nu, v, Jv
    log(f"matvec {mv_ms:.4f} ms at a fixed eps, {mv_red_ms:.4f} ms with the eps reduction and its read-back")

    # ---- warmup steps (the cylinder starts from rest: its warmup steps ramp
    # dt geometrically from dt/100 up to dt)
    for i in range(args.warmup):
        dti = dt
        if curved:
            dti = dt * 0.01 ** (1.0 - i / max(1, args.warmup - 1)) if args.warmup > 1 else dt * 0.01
        st = ctx.sdirk_step(u, dti)     # rebuilds the preconditioner when dt a^mm changes
        log(f"warmup step {i} (dt {dti:.4g}): newton {st['newton_its']} gmres {st['gmres_its']} "
            f"{st['t_total_ms']:.1f} ms")

    # ---- timed steps: a preconditioner build then K steps
    u_start = u.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tb0 = time.perf_counter()
    ctx.precond_build(u, dt_a)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb0) * 1e3
    stats = []
    evals = 0
    for i in range(args.steps):
        st = ctx.sdirk_step(u, dt)
        stats.append(st)
        evals += st["residual_evals"]
        log(f"step {i}: newton {st['newton_its']} gmres {st['gmres_its']} {st['t_total_ms']:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps

    # ---- dominant kernel: BRJ sweep (block-inverse GEMV + off-diagonal product)
    q = R.clone()
    o = ctx.empty()
    sweep_ms = time_apply(ctx, q, o, stream, max(3, args.kernel_reps // 20), cfg.brj_sweeps)
    sb = sweep_bytes(ctx, cfg, cfg.pc_precision)
    achieved = sb / (sweep_ms * 1e-3) / 1e9
    log(f"BRJ sweep {sweep_ms:.4f} ms, {achieved:.0f} GB/s")

    out = {
        "metric": "DG residual DOFs/s + implicit-step time, mixed/learned vs plain FP64 @1e-8",
        "value": cfg.dofs() / (res_ms * 1e-3), "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg.name, "elements": mesh.n_elem, "P": cfg.P, "nq": cfg.nq, "dim": cfg.dim,
                   "dofs_per_var": cfg.dofs(), "unknowns": ctx.n_unknowns, "scheme": cfg.scheme,
                   "cfl": cfg.cfl, "dt": dt, "Re": cfg.Re, "Ma": cfg.Ma, "newton_rtol": cfg.newton_rtol,
                   "gmres": f"GMRES({cfg.gmres_restart}) rtol {cfg.gmres_rtol}, {cfg.ortho}",
                   "brj_sweeps": cfg.brj_sweeps, "pc_precision": cfg.pc_precision, "pc_freeze": cfg.pc_freeze,
                   "pc_refresh_its": cfg.pc_refresh_its,
                   "geometry": "curved isoparametric O-grid, no-slip wall + far field" if curved
                   else "periodic affine boxes"},
        "roofline": {"bound": "hbm", "kernel": "k_brj_sweep", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(cfg.pc_precision, cfg.name),
                     "bytes_per_launch": sb, "avg_launch_ms": sweep_ms},
        "residual_roofline": residual_roofline(cfg, mesh.n_elem, res_ms),
        "residual_kernel": {"kernel": "k_res_fused", "ms": res_ms, "dofs_per_s": cfg.dofs() / (res_ms * 1e-3),
                            "unknowns_per_s": ctx.n_unknowns / (res_ms * 1e-3), "workgroup": tuned[0],
                            "three_kernel_ms": res3_ms,
                            "three_kernel_workgroups": dict(zip(("volume", "face", "lift"), tuned3)),
                            "speedup_vs_three_kernel": res3_ms / res_ms},
        "matvec": {"ms": mv_ms, "dofs_per_s": cfg.dofs() / (mv_ms * 1e-3), "ms_with_eps_reduction": mv_red_ms},
        "delivered_residual_dofs_per_s": cfg.dofs() * evals / wall,
        "pc_build_ms": build_ms,
        "residual_evals": evals,
        "newton_its": [s["newton_its"] for s in stats],
        "gmres_its": [s["gmres_its"] for s in stats],
    }

    if not args.no_forms:
        out["forms"] = bench_forms(ctx, u, cfg, dt, stream, args.form_steps)
        ctx.close()
        del ctx, q, o, R
        torch.cuda.empty_cache()
        if args.workload != 2:
            out["forms_tgv3d-16c-p3"] = bench_forms_tgv(args)

    if args.explicit:
        out["explicit_erk2"] = bench_explicit(cfg, mesh, u_start, u, wall * 1e3, args.steps * dt, kinds, states)
    del u_start

    if not args.no_learned:
        lcfg = W.config(args.learned_workload)
        out["learned"] = bench_learned(lcfg, lambda prec: make(prec, lcfg, lcfg.mesh()), args.learned_train,
                                       args.learned_held, args.learned_epochs)

    if args.batch:
        out["batch"] = bench_batch(args.batch_steps)

    if args.mms:
        out["mms_steady"] = [bench_mms(P, args.mms_n) for P in (2, 3, 4)]

    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


def bench_forms(ctx, u_end, cfg, dt, stream, nsteps):
    """The precision forms on this workload's context: from the state after
    the timed steps, the blocks built and stored in FP64, FP32 and BF16 in
    turn, then nsteps steps each; steps (build excluded), the build, the
    sweep's rate on the form's block bytes, and the state difference against
    the FP64 form (device against device; the tests compare each form's step
    with the FP64 oracle)."""
    import torch
    dt_a = dt * _lam(cfg.scheme)
    forms = {}
    base = None
    for prec in ("f64", "f32", "bf16"):
        ctx.set_pc_precision(prec)
        uu = u_end.clone()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ctx.precond_build(uu, dt_a)
        torch.cuda.synchronize()
        bms = (time.perf_counter() - tb) * 1e3
        t = time.perf_counter()
        its, gits = [], []
        for _ in range(nsteps):
            st = ctx.sdirk_step(uu, dt)
            its.append(st["newton_its"])
            gits.append(st["gmres_its"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / nsteps
        if base is None:
            base = uu.clone()
        q, o = ctx.empty(), ctx.empty()
        q.copy_(u_end)
        sw_ms = time_apply(ctx, q, o, stream, 3, cfg.brj_sweeps)
        sw_gbs = sweep_bytes(ctx, cfg, prec) / (sw_ms * 1e-3) / 1e9
        forms[prec] = {"ms_per_step": ms, "build_ms": bms, "newton_its": its, "gmres_its": gits,
                       "rel_diff_vs_f64_device": float(torch.linalg.vector_norm(uu - base) /
                                                       torch.linalg.vector_norm(base)),
                       "sweep_ms": sw_ms, "sweep_GBps": sw_gbs, "sweep_frac_hbm": sw_gbs / HBM_PEAK_GBS,
                       "sweep_traffic": measured_traffic(prec, cfg.name)}
        del q, o, uu
        log(f"form {prec}: build {bms:.1f} ms, {ms:.1f} ms/step, newton {its}, sweep {sw_ms:.4f} ms "
            f"{sw_gbs:.0f} GB/s")
    for prec in forms:
        forms[prec]["speedup_vs_f64"] = forms["f64"]["ms_per_step"] / forms[prec]["ms_per_step"]
    ctx.set_pc_precision(cfg.pc_precision)
    return forms


def bench_forms_tgv(args):
    """The precision forms on the 16^3 P = 3 Taylor-Green cube (SDIRK3 at
    CFL 20): 3 steps with each storage precision from the projected start."""
    import dataclasses
    import torch
    import workloads as W
    from paper_2002_04222_amd import Context
    cfg = W.config(2)
    mesh = cfg.mesh()
    dt = cfg.dt()
    forms = {}
    base = None
    q = None
    stream = torch.cuda.current_stream()
    for prec in ("f64", "f32", "bf16"):
        ctx = Context(mesh, cfg, pc_precision=prec)
        u = ctx.empty()
        ctx.project_tgv(torch.tensor(W.noise(ctx.shape, cfg.seed), dtype=torch.float64, device="cuda"),
                        cfg.noise_amp, u)
        if q is None:
            q = ctx.empty()
            ctx.residual(u, q)
        torch.cuda.synchronize()
        t = time.perf_counter()
        its = []
        for _ in range(3):
            its.append(ctx.sdirk_step(u, dt)["newton_its"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / 3
        if base is None:
            base = u.clone()
        o = ctx.empty()
        sw_ms = time_apply(ctx, q, o, stream, 5, cfg.brj_sweeps)
        sw_gbs = sweep_bytes(ctx, cfg, prec) / (sw_ms * 1e-3) / 1e9
        forms[prec] = {"ms_per_step": ms, "newton_its": its,
                       "rel_diff_vs_f64_device": float(torch.linalg.vector_norm(u - base) /
                                                       torch.linalg.vector_norm(base)),
                       "sweep_ms": sw_ms, "sweep_GBps": sw_gbs, "sweep_frac_hbm": sw_gbs / HBM_PEAK_GBS,
                       "sweep_traffic": measured_traffic(prec, cfg.name)}
        ctx.close()
        log(f"tgv3d form {prec}: {ms:.1f} ms/step (3 steps incl. the first build), sweep {sw_ms:.4f} ms "
            f"{sw_gbs:.0f} GB/s")
    for prec in forms:
        forms[prec]["speedup_vs_f64"] = forms["f64"]["ms_per_step"] / forms[prec]["ms_per_step"]
    return forms


def bench_explicit(cfg, mesh, u_start, u_impl, impl_ms, T, kinds, states):
    """The paper's implicit-versus-explicit comparison on this workload: the
    explicit ERK2 of Appendix A at its largest stable CFL (Eq. 32; found by
    bisection, a CFL counting as stable when, after 300 steps from the timed
    steps' start state, every value is finite and ||M^-1 L(u)|| has not grown
    past twice its start value: unstable modes are the highest ones, whose
    rate of change dominates that norm),
    timed over the same physical time T as the timed implicit steps (which
    include their preconditioner build), and the relative L2 difference of
    the two end states (the implicit run's temporal error at its CFL)."""
    import dataclasses
    import math
    import torch
    from paper_2002_04222_amd import Context
    ecfg = dataclasses.replace(cfg, scheme="erk2")
    ctx = Context(mesh, ecfg, bc_kind=kinds, bc_state=states)
    R = ctx.empty()

    def rate_norm(v):
        ctx.residual(v, R)
        return float(torch.linalg.vector_norm(R))

    r0 = rate_norm(u_start)
    dt20 = cfg.dt()                       # dt at cfg.cfl

    def stable(cfl, n=300):
        v = u_start.clone()
        dte = dt20 * cfl / cfg.cfl
        for _ in range(n):
            ctx.sdirk_step(v, dte)
        r = rate_norm(v)
        return math.isfinite(r) and r <= 2.0 * r0

    lo, hi = 0.01, 1.0
    if not stable(lo):
        ctx.close()
        return {"error": "ERK2 unstable at CFL 0.01"}
    for _ in range(8):
        mid = math.sqrt(lo * hi)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    cfl = lo
    for attempt in range(6):
        n_steps = int(math.ceil(T / (dt20 * cfl / cfg.cfl)))
        dte = T / n_steps
        v = u_start.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_steps):
            ctx.sdirk_step(v, dte)
        torch.cuda.synchronize()
        ems = (time.perf_counter() - t0) * 1e3
        diff = float(torch.linalg.vector_norm(v - u_impl) / torch.linalg.vector_norm(v))
        if math.isfinite(diff) and rate_norm(v) <= 2.0 * r0:
            break
        log(f"ERK2 at CFL {cfl:.4f} did not stay bounded over T; retrying at 0.8 x")
        cfl *= 0.8
    ctx.close()
    log(f"ERK2: largest stable CFL {cfl:.4f}, {n_steps} steps over T = {T:.4g} in {ems:.1f} ms; "
        f"implicit {impl_ms:.1f} ms; end states differ by {diff:.2e}")
    return {"cfl_max_stable": cfl, "cfl_implicit": cfg.cfl, "T": T, "explicit_steps": n_steps,
            "explicit_ms": ems, "implicit_ms": impl_ms, "implicit_speedup": ems / impl_ms,
            "rel_l2_diff_end_states": diff}


def bench_mms(P, n, drop=1e-8):
    """The paper's steady comparison on the manufactured Poiseuille flow
    (n x n elements on [0, 1]^2, Re 100, Ma 0.1, Dirichlet data from the exact
    solution): implicit SDIRK2 with the CFL number growing from 500 to 5000
    over the first ten steps and the blocks rebuilt every other step, against
    ERK2 at its largest stable CFL (bisection as in bench_explicit), each run
    from the uniform-velocity start until ||M^-1 L + s|| has dropped by
    `drop`.  Newton stops at alpha = 1e-3 (steady target; at 1e-8 Newton
    stalls at the rounding level of dt R once the state is nearly steady)."""
    import math
    import dataclasses
    import numpy as np
    import torch
    import workloads as W
    from paper_2002_04222_amd import Context
    cfg = W.mms_config(P, n)
    mesh = cfg.mesh()
    inp = W.mms_inputs(cfg, mesh)
    kinds, states = cfg.boundary()
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    def setup(scheme, **over):
        ctx = Context(mesh, dataclasses.replace(cfg, scheme=scheme), bc_kind=kinds, bc_state=states, **over)
        ctx.set_bc_field(dev(inp["bc_field"]))
        s = ctx.empty()
        ctx.project(dev(inp["forcing"]), s)
        ctx.set_source(s)
        u = ctx.empty()
        ctx.project(dev(inp["initial"]), u)
        return ctx, u

    R = None

    def rnorm(ctx, u):
        ctx.residual(u, R)
        return float(torch.linalg.vector_norm(R))

    ci, u = setup("sdirk2", pc_freeze=2, newton_rtol=1e-3)
    R = ci.empty()
    r0 = rnorm(ci, u)
    dt_cfl = cfg.dt() / cfg.cfl             # dt per unit CFL
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, newton, gmres = 0, 0, 0
    r = r0
    while r > drop * r0 and steps < 60:
        st = ci.sdirk_step(u, dt_cfl * 500.0 * 10.0 ** min(1.0, steps / 9.0))
        steps += 1
        newton += sum(st["newton_its"])
        gmres += sum(sum(x) for x in st["gmres_its"])
        r = rnorm(ci, u)
    torch.cuda.synchronize()
    impl_ms = (time.perf_counter() - t0) * 1e3
    ci.close()
    log(f"MMS P={P}: implicit steady in {steps} steps, {impl_ms:.0f} ms; ERK2 next")

    ce, u0 = setup("erk2")
    re0 = rnorm(ce, u0)

    def stable(cfl, k=2000, every=100):
        # on the way to a steady state ||M^-1 L + s|| decays; an unstable
        # mode makes it grow again
        v = u0.clone()
        best = re0
        for _ in range(k // every):
            for _ in range(every):
                ce.sdirk_step(v, dt_cfl * cfl)
            rr = rnorm(ce, v)
            if not math.isfinite(rr) or rr > 1.5 * best:
                return False
            best = min(best, rr)
        return True

    lo, hi = 0.005, 1.0
    for _ in range(8):
        mid = math.sqrt(lo * hi)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    cfl = lo
    for attempt in range(6):
        v = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        esteps = 0
        r = re0
        best = re0
        ok = True
        while r > drop * re0 and esteps < 3_000_000:
            for _ in range(500):
                ce.sdirk_step(v, dt_cfl * cfl)
            esteps += 500
            r = rnorm(ce, v)
            if not math.isfinite(r) or r > 1.5 * best:
                ok = False
                break
            best = min(best, r)
        torch.cuda.synchronize()
        expl_ms = (time.perf_counter() - t0) * 1e3
        if ok:
            break
        log(f"MMS P={P}: ERK2 at CFL {cfl:.4f} grew after {esteps} steps; retrying at 0.8 x")
        cfl *= 0.8
    ce.close()
    log(f"MMS P={P} {n}x{n}: implicit {steps} steps ({newton} Newton, {gmres} GMRES) {impl_ms:.0f} ms; "
        f"ERK2 CFL {cfl:.4f} {esteps} steps {expl_ms:.0f} ms; speed-up {expl_ms / impl_ms:.1f}")
    return {"P": P, "elements": mesh.n_elem, "implicit_steps": steps, "implicit_newton": newton,
            "implicit_gmres": gmres, "implicit_ms": impl_ms, "erk2_cfl_max_stable": cfl, "erk2_steps": esteps,
            "erk2_ms": expl_ms, "erk2_converged": ok, "implicit_speedup": expl_ms / impl_ms,
            "residual_drop": drop}


def bench_batch(steps):
    """64 independent 2D periodic Taylor-Green problems (N_x, N_y in 4..32,
    P in 2..5, Ma 0.1-0.5, Re 100-2000, SDIRK2 at CFL 20): SDIRK steps of the
    whole batch in lockstep against the same steps one instance at a time."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2002_04222_amd import Batch, Context
    cfgs = W.batch_configs(64, seed=5)
    dts = [c.dt() for c in cfgs]
    batch = Batch(cfgs)
    u = batch.empty()
    batch.project_tgv(torch.tensor(W.noise(batch.n_total, 5), device="cuda"), 1e-3, u)
    u0 = u.clone()
    tuned = batch.autotune(u, reps=5)
    log(f"batch autotuned residual workgroups per order group: {tuned}")
    R = batch.empty()
    for _ in range(3):
        batch.residual(u, R)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(10):
        batch.residual(u, R)
    torch.cuda.synchronize()
    res_ms = (time.perf_counter() - t) * 100.0
    batch.sdirk_step(u, dts)                       # warm-up (builds the preconditioners)
    torch.cuda.synchronize()
    t = time.perf_counter()
    its = []
    for _ in range(steps):
        ni, gi = batch.sdirk_step(u, dts)
        its.append(sum(sum(x) for x in gi))
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t) * 1e3 / steps
    log(f"batch: {batch_ms:.1f} ms per step of 64 instances, residual {res_ms:.3f} ms")
    # the same steps one instance at a time
    solo_ms = 0.0
    dofs = 0
    max_rel = 0.0
    for i, cfg in enumerate(cfgs):
        ctx = Context(cfg.mesh(), cfg, pc_refresh_its=0)   # the batch keeps the fixed freeze
        o = batch.offsets[i]
        ui = u0[o:o + batch.counts[i]].clone().reshape(ctx.shape)
        ctx.sdirk_step(ui, dts[i])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            ctx.sdirk_step(ui, dts[i])
        torch.cuda.synchronize()
        solo_ms += (time.perf_counter() - t) * 1e3 / steps
        a = ui.reshape(-1)
        b = u[o:o + batch.counts[i]]
        max_rel = max(max_rel, float((a - b).abs().max() / b.abs().max()))
        dofs += cfg.dofs()
        ctx.close()
    log(f"one by one: {solo_ms:.1f} ms per step of 64 instances")
    return {"instances": 64, "dofs_per_var": dofs, "unknowns": batch.n_total, "steps": steps,
            "ms_per_step_batched": batch_ms, "ms_per_step_one_by_one": solo_ms,
            "speedup": solo_ms / batch_ms, "residual_ms_batched": res_ms,
            "residual_dofs_per_s_batched": dofs / (res_ms * 1e-3),
            "gmres_its_per_step": its, "max_rel_diff_vs_one_by_one": max_rel,
            "autotuned_workgroups_per_group": tuned}


def bench_learned(cfg, make, n_train, held, epochs=150):
    """The learned-guess form: record n_train plain steps, fit the per-element
    MLP (its outputs averaged over the elements blend the increments'
    differences into the extrapolated guess) on the recorded stages (in the
    library), then from one saved state
    time `held` steps with each Newton initial guess (the paper's S_m, the
    extrapolated one, the learned one with its fallback), all stopping at the
    same absolute Newton tolerance."""
    import numpy as np
    import torch
    import workloads as W
    ctx, u = make("f64")
    dt = cfg.dt()
    n = ctx.n_unknowns
    stages = 2 if cfg.scheme == "sdirk2" else 3
    if cfg.geometry == "annulus":
        for i in range(5):                       # the cylinder's start: dt ramped from dt/100
            ctx.sdirk_step(u, dt * 0.01 ** (1.0 - i / 4.0))
    ctx.sdirk_step(u, dt)
    S_rec = torch.empty((n_train, stages, n), dtype=torch.float64, device="cuda")
    I_rec = torch.empty_like(S_rec)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(n_train):
        ctx.set_record(S_rec[k], I_rec[k])
        ctx.sdirk_step(u, dt)
        if (k + 1) % 10 == 0:
            log(f"learned: recorded {k + 1} of {n_train} steps")
    ctx.set_record(None, None)
    torch.cuda.synchronize()
    rec_s = time.perf_counter() - t
    nb = ctx.shape[1] * ctx.shape[2]
    ctx.mlp_create(256, W.mlp_init(2 * nb, 256, 2, seed=8))
    t = time.perf_counter()
    # in chunks of passes (the optimiser's state carries over between calls)
    done = 0
    while done < epochs:
        k = min(5, epochs - done)
        loss = ctx.mlp_fit(S_rec, I_rec, n_train, k, 1e-3)
        done += k
        log(f"learned: {done} of {epochs} passes, loss {loss:.3e}")
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t
    del S_rec, I_rec
    log(f"learned: recorded {n_train} steps in {rec_s:.1f} s, fit loss {loss:.3e} in {fit_s:.1f} s")
    u_save = u.clone()
    inc_save = torch.empty((3, stages, n), dtype=torch.float64, device="cuda")
    ctx.guess_state(inc_out=inc_save)
    res = {}
    for mode in ("paper", "extrapolated", "learned"):
        ctx.guess_state(inc_in=inc_save)
        ctx.set_guess(mode)
        uu = u_save.clone()
        ctx.precond_build(uu, dt * _lam(cfg.scheme))
        torch.cuda.synchronize()
        t = time.perf_counter()
        its, used, norms, blend = [], [], [], []
        for _ in range(held):
            st = ctx.sdirk_step(uu, dt)
            its.append(st["newton_its"])
            used.append(st["guess_used"])
            norms.append(st["guess_norm"])
            blend.append(st["guess_blend"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / held
        res[mode] = {"ms_per_step": ms, "newton_its": its, "u": uu, "used": used, "norms": norms, "blend": blend}
        log(f"guess {mode}: {ms:.1f} ms/step, newton {its}")
    ctx.set_guess("paper")
    base = res["paper"]["u"]
    out = {"train_steps": n_train, "epochs": epochs, "fit_loss": loss, "record_s": rec_s, "fit_s": fit_s,
           "held_out_steps": held}
    for mode, r in res.items():
        out[mode] = {"ms_per_step": r["ms_per_step"], "newton_its": r["newton_its"],
                     "guess_used": r["used"],
                     "guess_norm_N_S_extrap_learned": r["norms"] if mode != "paper" else None,
                     "learned_blend_c0_c1": r["blend"] if mode == "learned" else None,
                     "speedup_vs_paper_guess": res["paper"]["ms_per_step"] / r["ms_per_step"],
                     "rel_diff_vs_paper_guess": float(torch.linalg.norm(r["u"] - base) / torch.linalg.norm(base))}
    ctx.close()
    return out


def _lam(scheme):
    import numpy as np
    if scheme == "sdirk2":
        return 1.0 - np.sqrt(2.0) / 2.0
    lam = 0.4358665215
    for _ in range(20):
        lam -= (((lam - 3.0) * lam + 1.5) * lam - 1.0 / 6.0) / ((3.0 * lam - 6.0) * lam + 1.5)
    return lam


if __name__ == "__main__":
    main()
