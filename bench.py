#!/usr/bin/env python3
"""Grind-time benchmark of the five-equation RHS step on one MI355X.

Workload: the 3D air-water bubble cloud, 256^3 cells, two fluids (8 rows),
WENO5-JS + HLLC + SSP-RK3 at CFL 0.5, seeded synthetic initial condition.
One "step" is one SSP-RK3 step: a signal-speed reduction for dt and three RHS
evaluations (three axis passes each, the last fused with the stage update),
with the state resident in HBM.

Printed (one JSON line on stdout): FP64 grind time in ns per cell per RK stage
(`value`), the FP32 form's grind time, speedup and per-field error against the
FP64 path, the roofline of the dominant kernel (HIP events around every launch
on its own stream during the timed region), and the CPU oracle timed on this
host's cores on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grind time ns/cell/RK-stage FP64 vs FP32 + %HBM peak; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pass_bytes_per_cell(kind, neq, esize, ndim, stage_mix=(1, 1, 1)):
    """Algorithmic HBM bytes per cell of one launch of a pass kind.

    The passes of a stage run z, y, x (from the highest axis down): the first
    writes the RHS accumulator (read q, write acc), a middle one reads and
    writes it, and the x pass, last, reads q_k, acc and (stages 2 and 3) q^n
    and writes the next stage state.  In 1D the x pass is alone: q_k, q^n,
    next state.  The signal reduction reads q once.
    """
    first = {1: "pass_x", 2: "pass_y", 3: "pass_z"}[ndim]
    reads_qn = (0 + 1 + 1) / 3.0
    if kind == "signal":
        return neq * esize
    if kind == "pass_x":
        return ((2 if ndim == 1 else 3) + reads_qn) * neq * esize
    if kind == first:
        return 2 * neq * esize
    return 3 * neq * esize


# Algorithmic FP64 operations per cell for one axis pass of the 3D two-fluid
# system (counted from the method's formulas): cons->prim 21,
# WENO5-JS 97 per row x 8 rows, HLLC 106 per face, flux difference and
# volume-fraction source 30.  The stage update adds 32 per cell on the last pass.
FLOPS_PASS_3D2F = 21 + 97 * 8 + 106 + 30
FLOPS_STAGE_UPDATE = 32


def time_steps(S, q, steps, warmup, cfl, kernel_steps=None, repeats=1):
    """Wall time of `steps` CFL steps (HIP events on the stream, no per-launch
    instrumentation), as the median of `repeats` back-to-back loops, then
    per-kernel durations from the library's launch events over `kernel_steps`
    further steps (default: `steps`), in a loop of their own so that the
    event records do not inflate the step time.  Returns (median ms, kinds,
    every repeat's ms)."""
    import torch
    for _ in range(warmup):
        S.step(q, cfl=cfl)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    reps = []
    for _ in range(repeats):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(steps):
            S.step(q, cfl=cfl)
        t1.record(stream)
        torch.cuda.synchronize()
        reps.append(t0.elapsed_time(t1))
    ms = sorted(reps)[len(reps) // 2]
    S.set_timing(True)
    S.get_timing()
    for _ in range(steps if kernel_steps is None else kernel_steps):
        S.step(q, cfl=cfl)
    torch.cuda.synchronize()
    kinds = S.get_timing()
    S.set_timing(False)
    S.check()
    return ms, kinds, reps


def adjoint_cost(n=256, steps=200, every=20):
    """Forward vs forward+adjoint time of the adjoint problem (shock-cylinder
    physics, n x n, `steps` frozen-dt SSP-RK3 steps, checkpoints every `every`).

    J = time-integrated pressure of the last column; its gradient with respect
    to the initial alpha_1 and p goes through the hand-written adjoint.
    """
    import torch

    import workloads as W
    from paper_2503_07953_amd import autograd as AG
    from paper_2503_07953_amd.solver import Solver

    c = W.adjoint_case(n, steps=steps)
    S = Solver.from_case(c, precision="fp64")
    ex = c.extra
    t = lambda a: torch.from_numpy(a).cuda()

    def ic(alpha1, p):
        rows = [alpha1 * t(ex["rho_water"]), (1 - alpha1) * t(ex["rho_air"]), t(ex["u"]), t(ex["v"]), p,
                alpha1, 1 - alpha1]
        return torch.stack(rows).reshape(7, 1, n, n).contiguous()

    a0, p0 = t(c.w[5, 0].copy()), t(c.w[4, 0].copy())
    dt = 0.5 / S.max_signal(S.prim_to_cons(ic(a0, p0))).item()

    def run(grad):
        a = a0.clone().requires_grad_(grad)
        p = p0.clone().requires_grad_(grad)
        q = AG.PrimToCons.apply(ic(a, p), S)
        J = AG.rollout_objective(q, S, steps, dt, every=every)
        if grad:
            J.backward()
        return J

    run(False)
    torch.cuda.synchronize()
    t0 = time.time()
    run(False)
    torch.cuda.synchronize()
    tf = time.time() - t0
    run(True)
    torch.cuda.synchronize()
    t0 = time.time()
    run(True)
    torch.cuda.synchronize()
    tfb = time.time() - t0
    S.check()
    return {"workload": f"shock-cylinder adjoint problem {n}^2, {steps} frozen-dt steps, checkpoints every {every}",
            "forward_s": round(tf, 4), "forward_plus_adjoint_s": round(tfb, 4),
            "adjoint_over_forward": round((tfb - tf) / tf, 3), "total_over_forward": round(tfb / tf, 3)}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_bubble_cloud_256.md")


def _profile_data(path, tag, ncell):
    """The JSON line `tag` of a committed profile summary, or None when that
    summary was taken on different kernel sources (sha256 of the files it
    lists) or another size."""
    import hashlib
    try:
        line = next(l for l in open(path) if tag in l)
        data = json.loads(line.split(tag, 1)[1])
        h = hashlib.sha256()
        for src in data["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except (OSError, StopIteration, ValueError, KeyError):
        return None
    if h.hexdigest() != data.get("source_sha256") or data.get("cells") != ncell:
        return None
    return data


def measured_traffic_bytes(kind, prec, ncell):
    """Calibrated HBM bytes per launch of a sweep pass from the committed
    FETCH_SIZE / WRITE_SIZE summary (None if it is stale)."""
    data = _profile_data(TRAFFIC_FILE, "traffic-data:", ncell)
    return data.get("bytes_per_launch", {}).get(f"{kind}_{prec}") if data else None


def stage_alg_bytes(neq, esize):
    """Algorithmic bytes per cell per RK stage: a stage reads q^(k) (and q^n
    for k >= 2) and writes q^(k+1), on average (8/3) N_eq sizeof(Real)."""
    return (8.0 / 3.0) * neq * esize


def roofline_of(kinds, neq, esize, ndim, ncell, prec=None):
    """Roofline of the kernel kind with the largest total time.  achieved =
    the algorithmic bytes of one RK stage per cell ((8/3) N_eq sizeof) times
    the cells one launch covers, over its average launch duration (HIP events
    on the launch stream).  The pass's own implementation bytes (what the
    three-pass design must move in that launch) are reported beside it."""
    dom = max((k for k in kinds if kinds[k][1] > 0), key=lambda k: kinds[k][0])
    avg_ms = kinds[dom][0] / kinds[dom][1]
    bpc = stage_alg_bytes(neq, esize)
    achieved = bpc * ncell / (avg_ms * 1e-3) / 1e9
    impl = pass_bytes_per_cell(dom, neq, esize, ndim)
    tb = measured_traffic_bytes(dom, prec, ncell) if prec else None
    traffic = round(tb / (avg_ms * 1e-3) / 1e9, 1) if tb else None
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "avg_launch_ms": round(avg_ms, 5),
            "alg_bytes_per_cell": round(bpc, 2),
            "impl_bytes_per_cell": round(impl, 2),
            "impl_frac": round(impl * ncell / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic_bytes_per_cell": round(tb / ncell, 1) if tb else None}


VALU_FILE = os.path.join(ROOT, "profiles", "valu_sweep_bubble_cloud_256_fp64.md")
# FP64 vector rate of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# lane-operations per second (78.6 TFLOP/s counts an FMA as two flops); the
# same SIMDs issue 614.4 G wave64 instructions per second (4 cycles each).
FP64_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9
WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4


def measured_valu(kind, ncell):
    """VALU wave-instructions per launch of a sweep pass (counter summary;
    None if it is stale)."""
    data = _profile_data(VALU_FILE, "valu-data:", ncell)
    return data.get("valu_wave_instr_per_launch", {}).get(kind) if data else None


def field_group_errors(a, b, nf, ndim):
    """Max-relative L-inf and relative L2 error of a against b per conservative
    field (each partial density, the momentum vector, the energy, each alpha)."""
    import numpy as np
    groups = [[i] for i in range(nf)] + [list(range(nf, nf + ndim))] + [[nf + ndim]] + \
        [[nf + ndim + 1 + j] for j in range(nf if nf > 1 else 0)]
    linf, l2 = [], []
    for g in groups:
        da = np.sqrt(((a[g] - b[g]) ** 2).sum(axis=0))
        nb = np.sqrt((b[g] ** 2).sum(axis=0))
        linf.append(float(f"{da.max() / nb.max():.3e}"))
        l2.append(float(f"{np.linalg.norm(da) / np.linalg.norm(nb):.3e}"))
    return linf, l2


def periodic_slab_leg(n=512, steps=100, warmup=2):
    """The periodic air-water slab, n^3, `steps` CFL steps in the FP32 form and
    on the FP64 path: grind time, dominant-kernel roofline, FP32 error."""
    import torch

    import workloads as W
    from paper_2503_07953_amd.solver import Solver
    t_ic = time.time()
    c = W.periodic_slab(n, steps=steps)
    log(f"initial condition {c.name}: {time.time() - t_ic:.1f}s")
    out = {"workload": f"periodic air-water slab {n}^3, k^-2 velocity at rms Mach 0.3, {steps} CFL steps"}
    finals = {}
    for prec, esize in (("fp64", 8), ("fp32", 4)):
        S = Solver.from_case(c, precision=prec)
        q = S.prim_to_cons(S.to_device(c.w))
        q0 = q.clone()
        for _ in range(warmup):     # warm-up steps, then restart from the initial state
            S.step(q, cfl=c.cfl)
        q.copy_(q0)
        del q0
        ms, kinds, _ = time_steps(S, q, steps, 0, c.cfl, kernel_steps=10)
        g = ms / steps * 1e6 / (c.ncell * 3)
        out[prec] = {"ns_per_cell_stage": round(g, 5), "ms_per_step": round(ms / steps, 4),
                     "roofline": roofline_of(kinds, c.neq, esize, 3, c.ncell, prec)}
        finals[prec] = q.double().cpu().numpy()
        log(f"slab {prec}: {out[prec]}")
        del S, q
        torch.cuda.empty_cache()
    out["fp32_speedup_vs_fp64"] = round(out["fp64"]["ns_per_cell_stage"] / out["fp32"]["ns_per_cell_stage"], 3)
    linf, l2 = field_group_errors(finals["fp32"], finals["fp64"], 2, 3)
    out["fp32_error_vs_fp64"] = {"after_steps": steps + 10,
                                 "fields": ["alpha1 rho1", "alpha2 rho2", "momentum", "rho E", "alpha1", "alpha2"],
                                 "linf": linf, "l2": l2}
    del finals
    return out


def paper_shape_grind(steps=20, warmup=3):
    """The paper's single-device benchmark shape (Sec. 4.3.2: 3D, two fluids, 8
    PDEs) at 158^3 and 200^3 cells, from the bubble-cloud generator (seed 5):
    FP64 and FP32 grind, also per PDE (the paper's unit), each the median of
    three runs of warmup + steps CFL steps from the initial state."""
    import workloads as W
    from paper_2503_07953_amd.solver import Solver
    out = {}
    for n in (158, 200):
        c = W.bubble_cloud(n, seed=5)
        row = {}
        for prec in ("fp64", "fp32"):
            S = Solver.from_case(c, precision=prec)
            reps = []
            for _ in range(3):
                q = S.prim_to_cons(S.to_device(c.w))
                ms, _, _ = time_steps(S, q, steps, warmup, c.cfl, kernel_steps=0, repeats=1)
                reps.append(ms)
                del q
            g = sorted(reps)[1] / steps * 1e6 / (c.ncell * 3)
            row[f"{prec}_ns_per_cell_stage"] = round(g, 5)
            row[f"{prec}_ns_per_pde_stage"] = round(g / 8, 6)
            del S
        out[f"{n}^3"] = row
    return out


def variant_grind(case, variant, steps=20, warmup=3, riemann=0, low_mach=0, model=0, faces=None):
    """The same bubble cloud with the WENO5-Z (1) or TENO5 (2) weights of
    Sec. 4.2.2, the mapped WENO5-M weights (3) of Sec. 3.2.1, (riemann=1) the
    HLL face solver of Sec. 3.2.2, a low-Mach treatment (1 Thornber, 2 APC),
    Kapila's K (model=1) or a non-uniform grid (faces): FP64 and FP32 grind.
    A step that meets c^2 <= 0 is reported instead of a time."""
    import dataclasses

    from paper_2503_07953_amd import _lib as L
    from paper_2503_07953_amd.solver import Solver
    cz = dataclasses.replace(case, weno_variant=variant, riemann=riemann, low_mach=low_mach, model=model,
                             faces=faces)
    out = {}
    for prec in ("fp64", "fp32"):
        S = Solver.from_case(cz, precision=prec)
        reps = []
        try:
            for _ in range(3):
                # every repeat from the initial state: warmup + steps CFL steps
                q = S.prim_to_cons(S.to_device(cz.w))
                ms, _, _ = time_steps(S, q, steps, warmup, cz.cfl, kernel_steps=0, repeats=1)
                reps.append(ms)
                del q
        except L.MfcError as e:
            out[f"{prec}_ns_per_cell_stage"] = None
            out[f"{prec}_error"] = str(e)
            del S
            continue
        ms = sorted(reps)[1]
        out[f"{prec}_ns_per_cell_stage"] = round(ms / steps * 1e6 / (cz.ncell * 3), 5)
        del S
    return out


def shock_cylinder_grind(n=512, steps=100, warmup=5):
    import torch

    import workloads as W
    from paper_2503_07953_amd.solver import Solver
    c = W.shock_cylinder(n)
    S = Solver.from_case(c, precision="fp64")
    q = S.prim_to_cons(S.to_device(c.w))
    ms, _, _ = time_steps(S, q, steps, warmup, c.cfl, kernel_steps=0, repeats=3)
    return round(ms / steps * 1e6 / (c.ncell * 3), 5)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--repeats", type=int, default=1,
                    help="timed loops of --steps steps; the median is reported (default: exactly one loop)")
    ap.add_argument("--n", type=int, default=256, help="bubble-cloud grid edge (256 = the configuration)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (512^2 shock cylinder, reconstruction and face-solver variants, "
                         "the paper's 158^3 / 200^3 benchmark shape)")
    ap.add_argument("--no-slab", action="store_true", help="skip the 512^3 periodic-slab FP32/FP64 leg")
    ap.add_argument("--slab-n", type=int, default=512)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2503_07953_amd.solver import Solver

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {a.numel() * 8} bytes read and written")
        del a, b
    t_ic = time.time()
    case = W.bubble_cloud(args.n)
    log(f"initial condition {case.name}: {time.time() - t_ic:.1f}s")
    ncell = case.ncell
    neq = case.neq
    cfl = case.cfl

    # ---------------- FP64 ----------------
    S = Solver.from_case(case, precision="fp64")
    q = S.prim_to_cons(S.to_device(case.w))
    ms, kinds, reps = time_steps(S, q, args.steps, args.warmup, cfl, repeats=args.repeats)
    ms_step = ms / args.steps
    grind = ms_step * 1e6 / (ncell * 3)
    log(f"fp64: {ms_step:.3f} ms/step, {grind:.4f} ns/cell/stage, kinds {kinds}")

    # dominant kernel roofline: HBM on algorithmic bytes, the FP64 vector
    # units on algorithmic operations and (counters) on executed instructions,
    # and the attainable fraction: the larger of the two floors over the time
    roofline = roofline_of(kinds, neq, 8, case.ndim, ncell, "fp64")
    dom, avg_ms = roofline["kernel"], roofline["avg_launch_ms"]
    flops_cell = FLOPS_PASS_3D2F + (FLOPS_STAGE_UPDATE if dom == "pass_x" else 0)
    tflops = flops_cell * ncell / (avg_ms * 1e-3) / 1e12
    roofline["fp64_tflops_alg"] = round(tflops, 3)
    roofline["fp64_frac_alg"] = round(flops_cell * ncell / (avg_ms * 1e-3) / FP64_LANE_INSTR_PER_S, 4)
    t_valu_floor = flops_cell * ncell / FP64_LANE_INSTR_PER_S
    t_hbm_floor = stage_alg_bytes(neq, 8) * ncell / (HBM_PEAK_GBS * 1e9)
    roofline["attainable_frac"] = round(max(t_valu_floor, t_hbm_floor) / (avg_ms * 1e-3), 4)
    vi = measured_valu(dom, ncell)
    roofline["valu_issue_frac_counters"] = round(vi / (avg_ms * 1e-3) / WAVE_INSTR_PER_S, 4) if vi else None
    stage_bytes = stage_alg_bytes(neq, 8)  # per cell-stage, ideal fused path
    # whole stage: algorithmic operations of the three passes and the update
    stage_ms = ms_step / 3.0
    stage_ops = 3 * FLOPS_PASS_3D2F + FLOPS_STAGE_UPDATE
    stage_attainable = max(stage_ops * ncell / FP64_LANE_INSTR_PER_S,
                           stage_bytes * ncell / (HBM_PEAK_GBS * 1e9)) / (stage_ms * 1e-3)

    # ---------------- FP32 form ----------------
    fp32 = None
    if not args.no_fp32:
        S32 = Solver.from_case(case, precision="fp32")
        q32 = S32.prim_to_cons(S32.to_device(case.w))
        ms32, kinds32, _ = time_steps(S32, q32, args.steps, args.warmup, cfl, repeats=args.repeats)
        g32 = ms32 / args.steps * 1e6 / (ncell * 3)
        linf, l2 = field_group_errors(q32.double().cpu().numpy(), q.cpu().numpy(), 2, 3)
        fp32 = {"ns_per_cell_stage": round(g32, 5), "speedup_vs_fp64": round(grind / g32, 3),
                "steps_compared": args.warmup + (args.repeats + 1) * args.steps,
                "fields": ["alpha1 rho1", "alpha2 rho2", "momentum", "rho E", "alpha1", "alpha2"],
                "error_vs_fp64_linf": linf, "error_vs_fp64_l2": l2}
        log(f"fp32: {g32:.4f} ns/cell/stage, speedup {grind / g32:.2f}, linf {linf}")
        del S32, q32

    # ---------------- adjoint cost and the 2D configuration ----------------
    adj = None
    if not args.no_adjoint:
        adj = adjoint_cost()
        log(f"adjoint: {adj}")
    extra = None
    if not args.no_extra:
        extra = {"shock_cylinder_512_fp64_ns_per_cell_stage": shock_cylinder_grind(),
                 "bubble_cloud_weno_z": variant_grind(case, 1, args.steps, args.warmup),
                 "bubble_cloud_teno5": variant_grind(case, 2, args.steps, args.warmup),
                 "bubble_cloud_weno_m": variant_grind(case, 3, args.steps, args.warmup),
                 # the 256^3 bubble cloud breaks down under HLL at step index 26 (both the
                 # oracle and the library): this leg runs a fixed 3 + 20 steps
                 "bubble_cloud_hll": variant_grind(case, 0, 20, 3, riemann=1),
                 "bubble_cloud_low_mach": variant_grind(case, 0, args.steps, args.warmup, low_mach=1),
                 "bubble_cloud_apc": variant_grind(case, 0, args.steps, args.warmup, low_mach=2),
                 "bubble_cloud_kapila": variant_grind(case, 0, args.steps, args.warmup, model=1),
                 # centre-clustered grid, width ratio 2 along every axis
                 "bubble_cloud_stretched": variant_grind(
                     case, 0, args.steps, args.warmup,
                     faces=tuple(W.stretched_faces(args.n, 1.0, -1.0 / 3.0) for _ in range(3))),
                 "paper_benchmark_shape": paper_shape_grind(args.steps, args.warmup)}
        log(f"extra: {extra}")
    slab = None
    if not args.no_slab:
        del S
        torch.cuda.empty_cache()
        slab = periodic_slab_leg(args.slab_n)

    # ---------------- CPU oracle on this host ----------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        O = oracle.Oracle(case)
        qh = O.prim_to_cons(case.w)
        t0 = time.time()
        O.step(qh, cfl=cfl)
        t_cpu = time.time() - t0
        threads = oracle.num_threads()
        model = "unknown CPU"
        try:
            with open("/proc/cpuinfo") as f:
                model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
        except (OSError, StopIteration):
            pass
        del qh, O
        # the shock-cylinder configuration (512^2, 2D) on all threads: 20 steps
        c1 = W.shock_cylinder(512)
        O1 = oracle.Oracle(c1)
        q1 = O1.prim_to_cons(c1.w)
        t0 = time.time()
        O1.run(q1, 20, cfl=c1.cfl)
        t_c1 = time.time() - t0
        del q1, O1
        # one thread: 1 SSP-RK3 step of the same bubble-cloud generator at 64^3
        # (the per-cell work does not depend on the grid size)
        c64 = W.bubble_cloud(64, nbub=8, slab=8)
        O64 = oracle.Oracle(c64)
        q64 = O64.prim_to_cons(c64.w)
        oracle.set_num_threads(1)
        t0 = time.time()
        O64.step(q64, cfl=c64.cfl)
        t_1 = time.time() - t0
        oracle.set_num_threads(threads)
        cpu = {"value": round(t_cpu * 1e9 / (ncell * 3), 3), "unit": "ns/cell/RK-stage", "cores": threads,
               "kind": "oracle", "sample": f"1 SSP-RK3 step (3 RHS evaluations) of the {args.n}^3 bubble cloud, "
                                           f"{t_cpu:.1f} s wall on {threads} OpenMP threads ({model})",
               "shock_cylinder_512": {"value": round(t_c1 * 1e9 / (c1.ncell * 3 * 20), 3), "cores": threads,
                                      "sample": f"20 SSP-RK3 steps of the 512^2 shock-cylinder, {t_c1:.1f} s"},
               "single_thread": {"value": round(t_1 * 1e9 / (c64.ncell * 3), 3), "cores": 1,
                                 "sample": f"1 SSP-RK3 step of the 64^3 bubble cloud (8 bubbles), {t_1:.1f} s"}}
        log(f"cpu oracle: {cpu}")

    out = {
        "metric": METRIC, "value": round(grind, 5), "unit": "ns/cell/RK-stage", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded bubble-cloud initial condition)",
        "config": {"workload": f"3D air-water bubble cloud {args.n}^3, 64 bubbles, 100 bar pulse, "
                               f"2 fluids / 8 rows, WENO5-JS+HLLC+SSP-RK3, CFL 0.5",
                   "cells": ncell, "rows": neq},
        "repeats": args.repeats,
        "value_min_max": [round(min(reps) / args.steps * 1e6 / (ncell * 3), 5),
                          round(max(reps) / args.steps * 1e6 / (ncell * 3), 5)],
        "grind_ns_per_cell_pde_rhs": round(grind / neq, 6),
        "hbm_frac_stage_alg": round(stage_bytes / (grind * 1e-9) / 1e9 / HBM_PEAK_GBS, 4),
        "attainable_frac_stage": round(stage_attainable, 4),
        "kernel_ms": {k: [round(v[0], 4), v[1]] for k, v in kinds.items()},
        "roofline": roofline,
        "fp32_form": fp32,
        "adjoint_cost": adj,
        "other_workloads": extra,
        "periodic_slab": slab,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
