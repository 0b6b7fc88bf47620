"""Benchmark: time-to-solve at ||b - A x|| / ||b|| <= 1e-8 on one MI355X, per solver mode, with
the HBM roofline fraction of the dominant kernel and the CPU oracle as a reported baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config n1280_2560x1920x70] [--modes fp64,fp32_ir,...]

A step solves A x = b once in every listed mode (x0 = 0) on the 2560x1920x70 grid: FP64, FP32
inner iterations with FP64 refinement, and the same with BF16 couplings, all with the vertical
tridiagonal preconditioner; `value` is the sum of these times-to-solve.  Inputs are generated
on the host from the seeded recipe, copied to HBM and the operator is built before the timed
region.  After the timed steps, each once (after one untimed solve): the same modes with the
red-black line-SOR preconditioner ("_sor" suffix: three sweeps, omega 1.5) and the learned
preconditioner's modes on the same grid; the paper's Table 1 comparison (DP against its MP
BiCGStab); the learned preconditioner against the tridiagonal one on its own workload
(640x480x70) for two training recipes; the stress case (1280x960x140); and the CPU oracle,
timed on the host while those legs run.  One JSON line is printed on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# Algorithmic HBM bytes per grid point of one launch (reads + writes of the arrays the kernel
# must touch once), by kernel and precision (fp64, fp32, bf16, fp16).
BYTES_PER_POINT = {
    "spmv": {0: 80, 1: 40, 2: 28, 3: 28},       # 6 couplings + margin + x + dot partner + y
    "thomas_p": {0: 64, 1: 32, 2: 32, 3: 32},   # 3 LU factors + r, p, v in + p, phat out
    "thomas_s": {0: 56, 1: 28, 2: 28, 3: 28},   # 3 LU factors + r, v in + s, shat out (16-bit modes use FP32 factors)
    # line-SOR modes: the same with the result written in colour-major order and q once more
    # (its colour-major copy for the half-sweeps)
    "thomas_p_cm": {0: 72, 1: 36, 2: 36, 3: 36},
    "thomas_s_cm": {0: 64, 1: 32, 2: 32, 3: 32},
    "update": {0: 64, 1: 32, 2: 32, 3: 32},     # x, phat, shat, s, t, rhat in + x, r out
    "residual": {0: 76},                        # 6 couplings + margin + x + b (FP64) + r (FP32)
}
# Red-black line SOR: algorithmic bytes of one half-sweep per grid point (half the columns
# update: rhs q, own x in and out, the three LU factors and four horizontal couplings; the other
# half's x is read once as neighbours), times 2 * sweeps - 1 half-sweeps per application (the
# first red half-sweep is the tridiagonal solve before it).  The first half-sweep reads no old x
# of its own and the last writes the other colour's values in grid order as well: over an
# application these balance.  The generic kernel (level counts other than 70) also parks the
# forward-sweep values in memory (+8 B FP64, +4 B FP32 per point), which is not counted.
SOR_HALF_BYTES = {0: 44, 1: 22, 2: 18, 3: 18}
KERNEL_IDS = {"thomas_p": [0], "spmv": [1, 3], "thomas_s": [2], "update": [4], "residual": [5], "sor": [6, 7]}
KERNEL_SYMBOL = {"spmv": "k_spmv", "thomas_p": "k_thomas", "thomas_s": "k_thomas", "update": "k_update",
                 "residual": "k_spmv", "sor": "k_sor_half", "thomas_p_cm": "k_thomas", "thomas_s_cm": "k_thomas"}
PREC_NAME = {0: "fp64", 1: "fp32", 2: "bf16", 3: "fp16"}

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE and WRITE_SIZE on the 2560x1920x70
# grid (`python bench.py --traffic-probe` under `rocprofv3 --pmc`), scaled by the same counters
# on a device copy of known size (FETCH_SIZE x 2, WRITE_SIZE x 1).  Valid while the kernels
# are unchanged since that measurement; see profiles/hbm_traffic_2560x1920x70.txt.  The 16-bit
# modes run the FP32 tridiagonal and update kernels.
_C = "n1280_2560x1920x70"
MEASURED_TRAFFIC = {(_C, "spmv_fp64"): 28.74e9, (_C, "spmv_fp32"): 14.67e9, (_C, "spmv_bf16"): 9.82e9,
                    (_C, "residual_fp64"): 27.35e9,
                    (_C, "thomas_p_fp64"): 22.02e9, (_C, "thomas_s_fp64"): 19.27e9, (_C, "update_fp64"): 22.02e9,
                    (_C, "thomas_p_fp32"): 11.01e9, (_C, "thomas_s_fp32"): 9.63e9, (_C, "update_fp32"): 11.01e9,
                    (_C, "thomas_p_bf16"): 11.01e9, (_C, "thomas_s_bf16"): 9.63e9, (_C, "update_bf16"): 11.01e9,
                    (_C, "thomas_p_cm_fp64"): 24.77e9, (_C, "thomas_s_cm_fp64"): 22.02e9,
                    (_C, "thomas_p_cm_fp32"): 12.39e9, (_C, "thomas_s_cm_fp32"): 11.01e9,
                    (_C, "thomas_p_cm_bf16"): 12.39e9, (_C, "thomas_s_cm_bf16"): 11.01e9,
                    # one line-SOR application = five half-sweeps
                    (_C, "sor_fp64"): 81.75e9, (_C, "sor_fp32"): 40.24e9, (_C, "sor_bf16"): 32.78e9}


_T_START = time.perf_counter()


def log(*a):
    print(f"[{time.perf_counter() - _T_START:7.1f} s]", *a, file=sys.stderr, flush=True)


def generate_on_device(p, torch):
    import synth
    coef = torch.empty((7, p.nlev, p.nlat, p.nlon), dtype=torch.float64, device="cuda")
    for k, lev in synth.iter_coeff_levels(p, threads=16):
        coef[:, k].copy_(torch.from_numpy(lev))
    b = torch.empty(p.n, dtype=torch.float64, device="cuda")
    bv = b.view(p.nlev, p.nlat, p.nlon)
    for k in range(p.nlev):
        bv[k].copy_(torch.from_numpy(synth.rhs_level(p, k)))
    return coef, b


def copy_rate(torch, n: int) -> float:
    """GB/s of a device-to-device copy of n doubles (read + write), median of 5, HIP events."""
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    c = torch.empty_like(a)
    c.copy_(a)
    times = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        c.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    del a, c
    torch.cuda.empty_cache()
    times.sort()
    return round(2 * 8 * n / (times[2] * 1e-3) / 1e9, 1)


def _cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), for the record beside the CPU timing."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(gpu_fp64_iterations: int, sample_iters: int = 5):
    """The oracle (single-threaded C, -O2, no FMA contraction) on the host: a full FP64 solve of
    the 96x72x20 problem, a full solve of the 640x480x70 problem with the OpenMP build of the
    same source (thread count recorded), and a timed sample of `sample_iters` iterations on the benchmark's
    own 2560x1920x70 grid, scaled to the GPU's FP64 iteration count (extrapolated); the
    640x480x70 figure of the same kind is kept as context.  Per-iteration time = (time of a
    `sample_iters`-iteration run - 2 x one matrix-vector product) / `sample_iters` (the run
    forms the initial and the final true residual besides its iterations)."""
    import numpy as np

    import oracle
    import synth

    def per_iteration(p, threads):
        coef = synth.make_coeffs(p, threads=threads)
        b = synth.make_rhs(p).ravel()
        t0 = time.perf_counter()
        oracle.apply(coef, b)
        t_apply = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, info = oracle.bicgstab(coef, b, tol=1e-30, maxit=sample_iters)
        t_run = time.perf_counter() - t0
        del coef, b
        return (t_run - 2 * t_apply) / sample_iters, t_run, info.iterations

    out = {"unit": "s", "cores": 1, "kind": "oracle", "cpu_model": _cpu_model(), "host_threads": os.cpu_count()}
    p1 = synth.CONFIGS["small_96x72x20"]
    c1 = synth.make_coeffs(p1)
    b1 = synth.make_rhs(p1).ravel()
    t0 = time.perf_counter()
    _, i1 = oracle.bicgstab(c1, b1, tol=1e-8)
    out["small_96x72x20_full_solve"] = {"seconds": round(time.perf_counter() - t0, 3), "iterations": i1.iterations,
                                        "true_rel_residual": i1.true_rel_residual}
    del c1, b1
    # 640x480x70: a full solve with the OpenMP build of the same oracle source (fixed-partition
    # sums, so the same result for any thread count); one thread would take minutes
    p2 = synth.CONFIGS["manufactured_640x480x70"]
    c2 = synth.make_coeffs(p2, threads=16)
    b2 = synth.make_rhs(p2).ravel()
    t0 = time.perf_counter()
    _, i2 = oracle.bicgstab(c2, b2, tol=1e-8, parallel=True)
    out["c2_640x480x70_full_solve_openmp"] = {"seconds": round(time.perf_counter() - t0, 2), "iterations": i2.iterations,
                                              "true_rel_residual": i2.true_rel_residual,
                                              "threads": int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())}
    del c2, b2
    it2, _, _ = per_iteration(synth.CONFIGS["manufactured_640x480x70"], 16)
    out["context_640x480x70_seconds_per_iteration"] = round(it2, 3)
    it3, t_run, nits = per_iteration(synth.CONFIGS["n1280_2560x1920x70"], 8)
    out["n1280_seconds_per_iteration"] = round(it3, 2)
    out["value"] = round(it3 * gpu_fp64_iterations, 1)
    out["sample"] = (f"oracle FP64 BiCGStab + T^-1 on the 2560x1920x70 grid itself: a {nits}-iteration run took "
                     f"{t_run:.1f} s (1 thread), {it3:.2f} s per iteration after the two true-residual products; "
                     f"value = that x the GPU's FP64 iteration count ({gpu_fp64_iterations}): extrapolated, not a full "
                     f"CPU solve; timed on the host while the GPU legs after the timed steps ran")
    return out


def train_error_recipe(eg, torch, nops=100, nsnap=20, nval=10, epochs=20, lr=1e-3, batch=16, seed=1):
    """The learned preconditioner's configured recipe: (r_i, e_i = x* - x_i) pairs from the
    first nsnap iterates of FP64 BiCGStab solves (eg_harvest) on nops operators of the
    96x72x20 recipe with fresh perturbation seeds (1000 + s) and right-hand sides (seed 2000 + s);
    the last nval operators' pairs are held out for validation; Adam on the error-space loss
    ||M(r) - e||^2 / ||e||^2."""
    import synth
    t0 = time.perf_counter()
    ops, rs, es, owner = [], [], [], []
    for s in range(nops):
        p = synth.Problem(96, 72, 20, seed=1000 + s)
        op = eg.Operator(torch.from_numpy(synth.make_coeffs(p, threads=16)).cuda())
        r, e = op.harvest(torch.from_numpy(synth.make_rhs(p, seed=2000 + s).ravel()).cuda(), nsnap)
        ops.append(op)
        rs.append(r)
        es.append(e)
        owner += [s] * r.shape[0]
    ntrain_ops = nops - nval
    ntr = sum(int(r.shape[0]) for r in rs[:ntrain_ops])
    r = torch.cat(rs).contiguous()
    e = torch.cat(es).contiguous()
    del rs, es
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    net = eg.Net(11)
    net.set_loss(eg.Net.LOSS_ERROR)
    rv, ev, ov = r[ntr:].contiguous(), e[ntr:].contiguous(), [o - ntrain_ops for o in owner[ntr:]]
    val0 = net.eval(ops[ntrain_ops:], rv, ev, ov)
    t0 = time.perf_counter()
    hist = net.train(ops[:ntrain_ops], r[:ntr].contiguous(), e[:ntr].contiguous(), owner[:ntr], epochs=epochs,
                     batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    val1 = net.eval(ops[ntrain_ops:], rv, ev, ov)
    for op in ops:
        op.close()
    info = {"recipe": "error", "shape": [96, 72, 20], "operators": nops, "iterates_per_solve": nsnap,
            "pairs_train": ntr, "pairs_validation": int(rv.shape[0]), "epochs": epochs, "batch": batch, "lr": lr,
            "loss": "||M(r) - e||^2 / ||e||^2",
            "loss_train_first_epoch": round(float(hist[0]), 4), "loss_train_last_epoch": round(float(hist[-1]), 4),
            "loss_validation_untrained": round(val0, 4), "loss_validation_trained": round(val1, 4),
            "harvest_seconds": round(t_harvest, 2), "train_seconds": round(t_train, 2)}
    del r, e, rv, ev
    torch.cuda.empty_cache()
    return net, info


def train_krylov_recipe(eg, torch, shape, nops, nvec, epochs, seed=1):
    """Second recipe: the FGMRES basis vectors (the vectors a Krylov method applies the
    preconditioner to) of `nops` operators of the recipe at `shape`, residual-space loss."""
    import synth
    t0 = time.perf_counter()
    ops, rs, owner = [], [], []
    for s in range(nops):
        p = synth.Problem(*shape, seed=1000 + s)
        op = eg.Operator(torch.from_numpy(synth.make_coeffs(p, threads=16)).cuda())
        r, _ = op.harvest_krylov(torch.from_numpy(synth.make_rhs(p, seed=2000 + s).ravel()).cuda(), nvec,
                                 errors=False)
        ops.append(op)
        rs.append(r)
        owner += [s] * r.shape[0]
    r = torch.cat(rs).contiguous()
    del rs
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    net = eg.Net(11)
    loss0 = net.eval(ops, r, r, owner)
    t0 = time.perf_counter()
    hist = net.train(ops, r, r, owner, epochs=epochs, batch=16, lr=2e-3, seed=seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    for op in ops:
        op.close()
    info = {"recipe": "krylov", "shape": list(shape), "operators": nops, "vectors_per_operator": nvec,
            "pairs": int(r.shape[0]), "epochs": epochs, "loss": "||A M(r) - r||^2 / ||r||^2",
            "loss_untrained": round(loss0, 4), "loss_last_epoch": round(float(hist[-1]), 4),
            "harvest_seconds": round(t_harvest, 2), "train_seconds": round(t_train, 2)}
    del r
    torch.cuda.empty_cache()
    return net, info


def _timed_solve(op, torch, b, x, tol, mode, reps):
    """One untimed solve, then `reps` timed ones (median); returns (seconds, info)."""
    x.zero_()
    op.solve(b, x, tol, 20000, mode)
    times, info = [], None
    for _ in range(reps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = op.solve(b, x, tol, 20000, mode)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    times.sort()
    return times[len(times) // 2], info


def learned_comparison(eg, torch, nets, cfg_name, tol, reps=3):
    """On the learned preconditioner's workload, in FP32 inner + FP64 refinement and in FP64:
    BiCGStab with T^-1 (the method without the network), flexible BiCGStab with each trained
    network (and the tridiagonal fallback), FGMRES(30) with T^-1 and with each network.  After
    one untimed solve, the BiCGStab rows are the median of `reps` timed solves, the slower FGMRES
    rows the median of three."""
    import synth
    p = synth.CONFIGS[cfg_name]
    coef, b = generate_on_device(p, torch)
    op = eg.Operator(coef)
    del coef
    torch.cuda.empty_cache()
    out = {"workload": f"{p.nlon}x{p.nlat}x{p.nlev}, b ~ N(0,1), tol {tol}", "case": cfg_name,
           "timing": f"after one untimed solve, BiCGStab rows: median of {reps} timed solves; FGMRES rows: median of 3"}
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    runs = [("bicgstab_tri", None, 0), ("fgmres_tri", None, 1)]
    for name in nets:
        runs += [(f"bicgstab_learned_{name}", name, 0), (f"fgmres_learned_{name}", name, 1)]
    for prec, plain, learned in (("fp32_ir", eg.FP32_IR, eg.LEARNED_FP32_IR), ("fp64", eg.FP64, eg.LEARNED_FP64)):
        for label, net_name, method in runs:
            op.attach(nets[net_name] if net_name else None)
            op.set_option("method", method)
            op.set_option("learned_method", method)
            sec, info = _timed_solve(op, torch, b, x, tol, learned if net_name else plain, reps if method == 0 else 3)
            key = f"{label}_{prec}"
            out[key] = {"seconds": round(sec, 4), "iterations": info.iterations, "outer_steps": info.outer_steps,
                        "fallbacks": info.fallbacks, "status": info.status, "true_rel_residual": info.true_rel_residual}
            log(f"learned comparison {key}: {out[key]}")
    for prec in ("fp32_ir", "fp64"):
        base = out[f"bicgstab_tri_{prec}"]["seconds"]
        for name in nets:
            for m in ("bicgstab", "fgmres"):
                e = out[f"{m}_learned_{name}_{prec}"]
                e["time_vs_bicgstab_tri"] = round(e["seconds"] / base, 3)
    op.attach(None)
    op.close()
    return out


def stress_leg(eg, torch, net, cfg_name, tol):
    """The stress case (1280x960x140, shift 1e-6, vertical diffusivity contrast 1e4): plain FP64
    BiCGStab with T^-1, FP64 with the line SOR, FP32 inner + FP64 refinement with the line SOR
    and the learned preconditioner in FP32 + refinement (flexible BiCGStab with its fallback);
    one timed solve each after the operator's copies are built; every mode's difference from
    the FP64 + line-SOR solution."""
    import synth
    p = synth.CONFIGS[cfg_name]
    t0 = time.perf_counter()
    coef, b = generate_on_device(p, torch)
    op = eg.Operator(coef)
    del coef
    torch.cuda.empty_cache()
    t_gen = time.perf_counter() - t0
    op.attach(net)
    op.set_option("learned_method", 0)
    # build the FP32 and line-SOR copies outside the timed solves
    q = torch.zeros(p.n, dtype=torch.float32, device="cuda")
    op.apply(q, torch.empty_like(q), eg.PREC_FP32)
    op.set_option("precond", 1)
    op.precond(q, torch.empty_like(q), eg.PREC_FP32)
    q64 = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    op.precond(q64, torch.empty_like(q64), eg.PREC_FP64)
    del q, q64
    out = {"workload": f"{p.nlon}x{p.nlat}x{p.nlev}, shift {p.shift:g}, vertical diffusivity contrast 1e4, b ~ N(0,1), "
                       f"tol {tol}", "case": cfg_name, "generate_seconds": round(t_gen, 2), "timing": "one solve each"}
    sols = {}
    for name, mode, pc in (("fp64_sor", eg.FP64, 1), ("fp64", eg.FP64, 0), ("fp32_ir_sor", eg.FP32_IR, 1),
                           ("learned_fp32_ir", eg.LEARNED_FP32_IR, 0)):
        op.set_option("precond", pc)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = op.solve(b, x, tol, 20000, mode)
        torch.cuda.synchronize()
        out[name] = {"seconds": round(time.perf_counter() - t0, 3), "iterations": info.iterations,
                     "outer_steps": info.outer_steps, "fallbacks": info.fallbacks, "status": info.status,
                     "true_rel_residual": info.true_rel_residual}
        sols[name] = x
        log(f"stress {name}: {out[name]}")
    ref = sols["fp64_sor"]
    nref = torch.linalg.vector_norm(ref).item()
    for name, x in sols.items():
        if name != "fp64_sor":
            out[name]["rel_diff_vs_fp64_sor"] = torch.linalg.vector_norm(x - ref).item() / nref
    op.attach(None)
    op.close()
    del sols, ref, x, b
    torch.cuda.empty_cache()
    return out


def gpu_small_fp64(eg, torch, reps=5):
    """FP64 time-to-solve on the 96x72x20 correctness grid (launch-bound; beside the CPU oracle's
    full solve of the same problem)."""
    import synth
    p = synth.CONFIGS["small_96x72x20"]
    coef = torch.from_numpy(synth.make_coeffs(p)).cuda()
    b = torch.from_numpy(synth.make_rhs(p).ravel()).cuda()
    op = eg.Operator(coef)
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    sec, info = _timed_solve(op, torch, b, x, 1e-8, eg.FP64, reps)
    op.close()
    return {"seconds": round(sec, 5), "iterations": info.iterations, "true_rel_residual": info.true_rel_residual}


def paper_study(eg, torch, op, b):
    """The paper's own measurement on its grid (Table 1, Sec. 4): BiCGStab with tri_sor in FP64
    (DP) and in the paper's mixed precision (MP: FP32 vectors and coefficients, FP64 solution
    and global sums, restart every 150 iterations), to R = 1e-3 and 1e-4, and the iteration
    counts of both as the tolerance tightens (the question of Fig. 1 and Fig. 3)."""
    op.set_option("profile", 0)
    op.set_option("precond", 1)
    op.set_option("sor_sweeps", 3)
    op.set_option("sor_omega", 1.5)
    x = torch.zeros_like(b)
    sweep = {}
    for tol in (1e-3, 1e-4, 1e-6, 1e-8):
        row = {}
        for name, mode in (("dp", eg.FP64), ("mp", eg.FP32_MP)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = op.solve(b, x, tol, 2000, mode)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            row[name] = {"seconds": round(dt, 4), "iterations": info.iterations, "status": info.status,
                         "true_rel_residual": info.true_rel_residual,
                         "ms_per_iteration": round(1e3 * dt / max(info.iterations, 1), 3)}
        sweep[f"{tol:g}"] = row
        log(f"paper study tol {tol:g}: {row}")
    op.set_option("precond", 0)
    table1 = {}
    for tol in ("0.001", "0.0001"):
        r = sweep[tol]
        table1[tol] = {"dp_seconds": r["dp"]["seconds"], "mp_seconds": r["mp"]["seconds"],
                       "dp_iterations": r["dp"]["iterations"], "mp_iterations": r["mp"]["iterations"],
                       "mp_over_dp_per_iteration": round(r["mp"]["ms_per_iteration"] / r["dp"]["ms_per_iteration"], 3),
                       "paper_mp_over_dp_per_iteration": {"0.001": 0.585, "0.0001": 0.573}[tol]}
    return {"preconditioner": "tri_sor as red-black line SOR, 3 sweeps, omega 1.5", "table1": table1,
            "tolerance_sweep": sweep}


def fig1_study(eg, torch, configs=("small_96x72x20", "manufactured_640x480x70"), tol=1e-10):
    """The paper's toy-model comparison (Sec. 4, Fig. 1): the all-32-bit BiCGStab (FP32 vectors,
    coefficients and solution, FP64 sums; EG_FP32_MP with option mp_x32, no periodic restarts)
    against the FP64 one, both with T^-1, R (the solver's recursive relative residual) against
    iteration.  For R_c = 1e-1 .. 1e-8: the first iteration at which each solver's R reaches R_c,
    their ratio, and the time to get there (iterations x that solver's time per iteration)."""
    import numpy as np
    import synth
    out = {}
    for name in configs:
        p = synth.CONFIGS[name]
        coef, b = generate_on_device(p, torch)
        op = eg.Operator(coef)
        del coef
        op.set_option("restart_every", 10 ** 9)
        rows, hist = {}, {}
        maxit = 20000
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        for label, mode, x32 in (("dp", eg.FP64, 0), ("sp", eg.FP32_MP, 1)):
            op.set_option("mp_x32", x32)
            x.zero_()
            op.solve(b, x, 1e-3, 50, mode)   # untimed: work vectors and coefficient copies
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = op.solve(b, x, tol, maxit, mode)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            h = np.asarray(op.history())
            hist[label] = h
            rows[label] = {"iterations": info.iterations, "status": info.status, "seconds": round(dt, 4),
                           "ms_per_iteration": round(1e3 * dt / max(info.iterations, 1), 4),
                           "true_rel_residual": info.true_rel_residual,
                           "min_recursive_R": float(h.min()) if h.size else None,
                           "R_every_5th_iteration": [float(f"{v:.3g}") for v in h[4::5]]}
            if label == "dp":
                maxit = 3 * info.iterations + 50
        op.set_option("mp_x32", 0)
        cross = {}
        for k in range(1, 9):
            e = {}
            for label in ("dp", "sp"):
                hit = np.nonzero(hist[label] <= 10.0 ** -k)[0]
                its = int(hit[0]) + 1 if hit.size else None
                e[f"{label}_iterations"] = its
                e[f"{label}_ms"] = round(its * rows[label]["ms_per_iteration"], 3) if its else None
            if e["dp_iterations"] and e["sp_iterations"]:
                e["sp_over_dp_iterations"] = round(e["sp_iterations"] / e["dp_iterations"], 3)
                e["sp_over_dp_time"] = round(e["sp_ms"] / e["dp_ms"], 3)
            cross[f"1e-{k}"] = e
        rows["by_R"] = cross
        rows["time_per_iteration_sp_over_dp"] = round(rows["sp"]["ms_per_iteration"] / rows["dp"]["ms_per_iteration"], 3)
        out[name] = rows
        log(f"fig1 study {name}: " + ", ".join(f"{rc}: {e.get('sp_over_dp_iterations')}" for rc, e in cross.items()))
        op.close()
        del b, x
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="n1280_2560x1920x70")
    ap.add_argument("--modes", default="fp64,fp32_ir,fp32_ir_bf16")
    ap.add_argument("--extra-modes", default="fp32_ir_fp16,fp64_sor,fp32_ir_sor,fp32_ir_bf16_sor,fp32_ir_fp16_sor,"
                                             "learned_fp32_ir",
                    help="modes timed once each after the timed steps ('' skips them)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--learned-config", default="learned_640x480x70",
                    help="workload of the learned-preconditioner comparison ('' skips it)")
    ap.add_argument("--learned-reps", type=int, default=5,
                    help="timed solves per BiCGStab row of the learned comparison (median; FGMRES rows: 3)")
    ap.add_argument("--stress-config", default="stress_1280x960x140", help="stress case ('' skips it)")
    ap.add_argument("--error-ops", type=int, default=100, help="96x72x20 operators of the error-loss recipe")
    ap.add_argument("--error-epochs", type=int, default=20)
    ap.add_argument("--train-shape", default="160x120x70")
    ap.add_argument("--train-ops", type=int, default=16)
    ap.add_argument("--train-vecs", type=int, default=20)
    ap.add_argument("--train-epochs", type=int, default=20)
    ap.add_argument("--no-paper-study", action="store_true",
                    help="skip the paper's comparisons (DP vs MP of its Table 1, 32- vs 64-bit of its Fig. 1)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run four iterations of each mode and a device copy of known size (for counter runs) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU decomposition "
              f"is not built in this framework", file=sys.stderr)
        sys.exit(2)

    import threading

    import numpy as np
    import torch

    import paper_1811_03852_amd as eg
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    p = synth.CONFIGS[args.config]
    if args.traffic_probe:
        traffic_probe(eg, torch, p, args)
        return
    name2mode = {v: k for k, v in eg.MODE_NAMES.items()}

    def parse_modes(text):
        # a "_sor" suffix runs the mode with the red-black line SOR preconditioner (option precond 1)
        out = []
        for m in text.split(","):
            if m:
                sor = m.endswith("_sor")
                out.append((m, name2mode[m[:-4] if sor else m], sor))
        return out

    runs = parse_modes(args.modes)
    extra = parse_modes(args.extra_modes)
    learned_modes = (eg.LEARNED_FP64, eg.LEARNED_FP32_IR)
    need_net = bool(args.learned_config or args.stress_config) or any(m in learned_modes for _, m, _ in runs + extra)

    nets, training = {}, {}
    if need_net:
        nets["error"], training["error"] = train_error_recipe(eg, torch, nops=args.error_ops,
                                                              epochs=args.error_epochs)
        log(f"trained the network (error recipe): {training['error']}")
        if args.learned_config:
            shape = tuple(int(v) for v in args.train_shape.split("x"))
            nets["krylov"], training["krylov"] = train_krylov_recipe(eg, torch, shape, args.train_ops, args.train_vecs,
                                                                     args.train_epochs)
            log(f"trained the network (Krylov recipe): {training['krylov']}")

    t0 = time.perf_counter()
    coef, b = generate_on_device(p, torch)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    log(f"generated {args.config} ({p.nlon}x{p.nlat}x{p.nlev}) in {t_gen:.1f} s")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = eg.Operator(coef)
    torch.cuda.synchronize()
    t_setup64 = time.perf_counter() - t0
    del coef
    torch.cuda.empty_cache()
    # build the lower-precision copies the modes need (timed separately from the solves)
    scratch = torch.zeros(p.n, dtype=torch.float32, device="cuda")
    out = torch.empty_like(scratch)
    t_setup_low = {}
    for _, m, _ in runs + extra:
        prec = {eg.FP32_IR: eg.PREC_FP32, eg.FP32_IR_BF16: eg.PREC_BF16, eg.FP32_IR_FP16: eg.PREC_FP16,
                eg.LEARNED_FP32_IR: eg.PREC_FP32}.get(m)
        if prec is not None and PREC_NAME[prec] not in t_setup_low:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            op.apply(scratch, out, prec)
            torch.cuda.synchronize()
            t_setup_low[PREC_NAME[prec]] = time.perf_counter() - t0
    del scratch, out

    if "error" in nets:
        op.attach(nets["error"])
    op.set_option("learned_method", 0)   # flexible BiCGStab, the method the configuration names
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        for name, m, sor in runs:
            op.set_option("precond", 1 if sor else 0)
            x.zero_()
            info = op.solve(b, x, args.tol, 20000, m)
            log(f"warmup {name}: {info}")

    op.set_option("profile", 1)
    op.reset_kernel_stats()
    stats = {}   # (kernel name, precision) -> [launches, total ms]

    def collect(sor):
        # the library's HIP-event times of the last solve; in the line-SOR modes the
        # tridiagonal kernels also write the colour-major copies (listed as *_cm)
        for kname, ids in KERNEL_IDS.items():
            key = f"{kname}_cm" if sor and kname in ("thomas_p", "thomas_s") else kname
            for prec in range(4):
                for kid in ids:
                    c, t = op.kernel_stats(kid, prec)
                    if c:
                        e = stats.setdefault((key, prec), [0, 0.0])
                        e[0] += c
                        e[1] += t
        op.reset_kernel_stats()

    per_mode = {name: {"seconds": [], "iterations": None, "outer_steps": None, "status": None,
                       "true_rel_residual": None} for name, _, _ in runs}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for step in range(args.steps):
        for name, m, sor in runs:
            op.set_option("precond", 1 if sor else 0)
            x.zero_()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            info = op.solve(b, x, args.tol, 20000, m)
            torch.cuda.synchronize()
            d = per_mode[name]
            d["seconds"].append(time.perf_counter() - ts)
            collect(sor)
            d.update(iterations=info.iterations, outer_steps=info.outer_steps, status=info.status,
                     true_rel_residual=info.true_rel_residual, fallbacks=info.fallbacks)
        log(f"timed step {step + 1}/{args.steps}: " + ", ".join(f"{k} {v['seconds'][-1]:.3f} s" for k, v in per_mode.items()))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1000.0 * elapsed / args.steps
    op.set_option("profile", 0)

    # per-kernel achieved bandwidth from the library's HIP-event timing over the timed region
    kernels = {}
    order = list(KERNEL_SYMBOL)
    for (kname, prec), (cnt, ms) in sorted(stats.items(), key=lambda kv: (order.index(kv[0][0]), kv[0][1])):
        if kname != "sor" and prec not in BYTES_PER_POINT[kname]:
            continue
        bpp = SOR_HALF_BYTES[prec] * (2 * 3 - 1) if kname == "sor" else BYTES_PER_POINT[kname][prec]
        bytes_launch = bpp * p.n
        avg_ms = ms / cnt
        kernels[f"{kname}_{PREC_NAME[prec]}"] = {
            "symbol": KERNEL_SYMBOL[kname], "launches": cnt, "avg_ms": round(avg_ms, 4),
            "total_ms": round(ms, 2), "bytes_per_launch": bytes_launch,
            "gbs": round(bytes_launch / (avg_ms * 1e-3) / 1e9, 1),
            "measured_bytes_per_launch": MEASURED_TRAFFIC.get((args.config, f"{kname}_{PREC_NAME[prec]}"))}
    dom_name = max(kernels, key=lambda k: kernels[k]["total_ms"])
    dom = kernels[dom_name]
    traffic = MEASURED_TRAFFIC.get((args.config, dom_name))
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": dom["gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(dom["gbs"] / PEAK_HBM_GBS, 4), "traffic": traffic,
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "bytes_per_launch": dom["bytes_per_launch"], "avg_ms": dom["avg_ms"],
                "copy_gbs": copy_rate(torch, p.n),
                "copy_note": "device-to-device copy of one FP64 grid vector on the same GPU, read + write bytes / "
                             "time (median of 5): the attainable streaming rate, context for frac, not its denominator"}

    modes_out = {}
    for k, d in per_mode.items():
        modes_out[k] = {"seconds": round(float(np.median(d["seconds"])), 4), "iterations": d["iterations"],
                        "outer_steps": d["outer_steps"], "status": d["status"],
                        "true_rel_residual": d["true_rel_residual"]}
    fp64_iters = per_mode.get("fp64", {}).get("iterations")

    # the CPU oracle runs on the host while the GPU legs below keep the GPU busy
    cpu = None
    cpu_thread = None
    if not args.no_cpu_baseline:
        box = {}

        def run_cpu():
            try:
                box["result"] = cpu_baseline(fp64_iters or 1)
            except Exception as exc:   # reported, not fatal to the GPU measurement
                box["result"] = {"error": repr(exc)}

        log("timing the CPU oracle on the host (background) ...")
        cpu_thread = threading.Thread(target=run_cpu, daemon=True)
        cpu_thread.start()

    # the other modes on the same grid, once each after an untimed solve
    extra_out = {}
    for name, m, sor in extra:
        op.set_option("precond", 1 if sor else 0)
        sec, info = _timed_solve(op, torch, b, x, args.tol, m, 1)
        extra_out[name] = {"seconds": round(sec, 4), "iterations": info.iterations, "outer_steps": info.outer_steps,
                           "fallbacks": info.fallbacks, "status": info.status,
                           "true_rel_residual": info.true_rel_residual}
        log(f"{args.config} {name}: {extra_out[name]}")
    op.set_option("precond", 0)
    paper = None if args.no_paper_study else paper_study(eg, torch, op, b)
    op.attach(None)
    op.close()
    del x, b
    torch.cuda.empty_cache()

    small = gpu_small_fp64(eg, torch)
    fig1 = None if args.no_paper_study else fig1_study(eg, torch)
    learned = None
    if args.learned_config:
        learned = learned_comparison(eg, torch, nets, args.learned_config, args.tol, args.learned_reps)
        learned["training"] = training
    stress = None
    if args.stress_config:
        stress = stress_leg(eg, torch, nets.get("error"), args.stress_config, args.tol)
    if cpu_thread is not None:
        cpu_thread.join()
        cpu = box["result"]
        if "small_96x72x20_full_solve" in cpu:
            cpu["small_96x72x20_gpu_fp64"] = small

    dtypes = sorted({{eg.FP64: "f64", eg.FP32_IR: "f64+f32", eg.FP32_IR_BF16: "f64+f32+bf16",
                      eg.FP32_IR_FP16: "f64+f32+f16", eg.LEARNED_FP64: "f64+bf16mfma",
                      eg.LEARNED_FP32_IR: "f64+f32+bf16mfma", eg.FP32_MP: "f64+f32"}[m] for _, m, _ in runs})
    result = {
        "metric": "time-to-solve at ||r||/||b||<=1e-8, FP64 vs mixed vs learned-PC; HBM GB/s",
        "value": round(ms_per_step / 1000.0, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ",".join(dtypes),
        "data": "synthetic (seeded operator recipe and b ~ N(0,1); no UM data)",
        "config": {"workload": f"{p.nlon}x{p.nlat}x{p.nlev} Helmholtz solve to 1e-8, one solve per mode "
                               f"({','.join(name for name, _, _ in runs)}); value = the sum of these times-to-solve",
                   "case": args.config, "grid": [p.nlon, p.nlat, p.nlev], "dof": p.n, "tol": args.tol,
                   "parallelism": "1 GPU"},
        "value_is": "sum over the step's modes of the time-to-solve (see modes for each)",
        "modes": modes_out,
        "other_modes": extra_out,
        "setup_seconds": {"generate_host": round(t_gen, 2), "operator_fp64": round(t_setup64, 3),
                          **{f"operator_{k}": round(v, 3) for k, v in t_setup_low.items()}},
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "learned": learned,
        "stress": stress,
        "paper_study": paper,
        "fig1_study": fig1,
    }
    print(json.dumps(result), flush=True)


def traffic_probe(eg, torch, p, args):
    """Four iterations of each mode, two line-SOR iterations of each, a device copy of known
    size, and three network applications on the learned preconditioner's workload in each of
    its two inference paths, for counter runs."""
    import synth
    coef, b = generate_on_device(p, torch)
    op = eg.Operator(coef)
    del coef
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    for m in (eg.FP64, eg.FP32_IR, eg.FP32_IR_BF16):
        x.zero_()
        op.solve(b, x, args.tol, 4, m)
    op.set_option("precond", 1)   # the line-SOR half-sweeps
    for m in (eg.FP64, eg.FP32_IR, eg.FP32_IR_BF16):
        x.zero_()
        op.solve(b, x, args.tol, 2, m)
    op.set_option("precond", 0)
    for _ in range(3):
        x.copy_(b)
    torch.cuda.synchronize()
    op.close()
    del x, b
    torch.cuda.empty_cache()
    # three network applications on the learned preconditioner's workload
    p4 = synth.CONFIGS[args.learned_config or "learned_640x480x70"]
    coef, _ = generate_on_device(p4, torch)
    op = eg.Operator(coef)
    del coef
    net = eg.Net(11)
    q = torch.randn(p4.n, dtype=torch.float32, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    for fused in (1, 0):   # the one-launch inference, then the layer-by-layer kernels
        op.set_option("net_fused", fused)
        for _ in range(3):
            net.apply(op, q)
    torch.cuda.synchronize()
    print(json.dumps({"traffic_probe": args.config, "copy_bytes_read": p.n * 8, "copy_bytes_written": p.n * 8,
                      "net_workload": args.learned_config or "learned_640x480x70"}))


if __name__ == "__main__":
    main()
