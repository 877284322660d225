"""Benchmark of the explicit RBF-FD Poisson iteration on one MI355X.

Workload: 3D unit cube, 100^3 jittered grid (jitter 0.3h, seed 1), Dirichlet
data from u = sin(pi x) sin(pi y) sin(pi z), PHS r^3 + monomials of order m
with n = 2*C(m+3, 3) nearest nodes (m = 4, n = 70 is the headline; m = 2 and 6
are reported beside it).  One step = one explicit sweep
u <- u + dt (L_h u - f) over all interior nodes (with the fused Dirichlet rows
and max-residual reduction), run by the library in HIP-graph chunks.

Prints one JSON line: node-updates/s (value), HBM GB/s of the sweep kernel
against the 8 TB/s peak (roofline), setup times, time to L-inf error 1e-6
for FP64 vs FP32+FP64 refinement on the 1M-node cube, the CPU oracle's
OpenMP sweep on the same operator as a baseline, the 8M-node cube's FP32 +
refinement vs FP64 step times (2,000 steps each), and the 2M-node adjoint
gradient against central differences on 32 directions and against the
oracle's transposed loop.  Inputs are synthetic and seeded; they are in HBM
before timing.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# MI355X FP64: 78.6 TFLOP/s dense, vector FMA and matrix cores alike
PEAK_FP64_FLOPS = 78.6e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def sweep_source_hash():
    """Hash of the sweep kernels' sources (the kernels and their row sums)."""
    h = hashlib.sha256()
    for name in ("k_sweep.hip", "row_dot.h"):
        with open(os.path.join(ROOT, "paper_2502_12878_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(key, shape):
    """HBM bytes per sweep launch measured with rocprofv3 counters, if they
    were taken on the current sweep source in the same sweep shape; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(key)
    if not e or e.get("kernel_source") != sweep_source_hash() or e.get("shape") != shape:
        return None
    return e.get("bytes_per_launch")


def setup_problem(m, keep_fp32=False, autotune=True):
    import torch

    import rbf_inputs as ri
    from paper_2502_12878_amd import Problem

    wl = ri.workload("cube1M", m=m)
    p = Problem(0)
    t0 = time.perf_counter()
    xyz, typ = p.build_nodes(wl.dim, wl.side, wl.jitter, wl.seed)
    p.set_nodes(xyz, typ)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p.build_stencils(wl.n)
    t2 = time.perf_counter()
    p.compute_weights(wl.m, keep_fp32=keep_fp32)
    t3 = time.perf_counter()
    if autotune:
        p.autotune()
    # manufactured problem (the generator's coordinates equal the GPU's bit for bit)
    xyz_h, typ_h = wl.nodes()
    u_ex, f, g, u0 = ri.manufactured(wl.dim, xyz_h, typ_h)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    return dict(p=p, wl=wl, f=dev(f), u0=dev(u0), u_ex=dev(u_ex), typ=typ_h, f_h=f, u0_h=u0,
                setup={"nodes_s": t1 - t0, "stencils_s": t2 - t1, "weights_s": t3 - t2})


def time_sweeps(s, steps, warmup, chunk=500):
    """Wall time of one call of `steps` explicit steps in graph chunks of
    min(chunk, steps), after untimed warm-up calls identical to it (so its
    graphs are built and cached before timing) covering at least `warmup`
    steps; also the device time per sweep (events around the chunk graphs)
    of the timed call.  Returns (wall s, s per sweep, sweeps timed, report,
    warm-up steps run)."""
    import torch
    p, wl = s["p"], s["wl"]
    chunk = max(1, min(chunk, steps))
    warm = 0
    while True:
        u = s["u0"].clone()
        st, _ = p.iterate(s["f"], u, wl.dt, steps, 0.0, chunk)
        assert st == 0, st
        warm += steps
        if warm >= warmup:
            break
    u = s["u0"].clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rep = p.iterate(s["f"], u, wl.dt, steps, 0.0, chunk)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert st == 0, (st, rep)
    per_sweep, nsw = p.last_sweep_time()
    return t1 - t0, per_sweep, nsw, rep, warm


def sweep_windows(s, windows=5, steps=1000, chunk=500):
    """Device time per sweep over `windows` further windows of `steps` steps
    (HIP events around the chunk graphs, which the timed call has already
    built): median, minimum and maximum, in ms per sweep."""
    import numpy as np
    import torch
    p, wl = s["p"], s["wl"]
    per = []
    for _ in range(windows):
        u = s["u0"].clone()
        st, _ = p.iterate(s["f"], u, wl.dt, steps, 0.0, chunk)
        assert st == 0, st
        per.append(1e3 * p.last_sweep_time()[0])
    torch.cuda.synchronize()
    return {"windows": windows, "steps_each": steps, "median_ms_per_sweep": round(float(np.median(per)), 5),
            "min_ms_per_sweep": round(min(per), 5), "max_ms_per_sweep": round(max(per), 5)}


def time_to_error(s, target, inner=500, max_steps=2_000_000):
    """Steps and device time until max|u - u_exact| <= target, plain FP64 vs
    FP32 inner sweeps with FP64 outer correction (checked every `inner` steps
    in both modes)."""
    import torch
    from paper_2502_12878_amd import RBF_MODE_FP64, RBF_MODE_MIXED
    p, wl = s["p"], s["wl"]
    out = {}
    finals = {}
    for name, mode in (("fp64", RBF_MODE_FP64), ("fp32_refine", RBF_MODE_MIXED)):
        u = s["u0"].clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, rep = p.iterate(s["f"], u, wl.dt, max_steps, 0.0, inner, mode=mode, inner_steps=inner,
                            u_ref=s["u_ex"], err_target=target)
        torch.cuda.synchronize()
        out[name] = {"status": st, "steps": rep["steps"], "wall_s": round(time.perf_counter() - t0, 3),
                     "device_s": round(rep["seconds"], 3), "err_inf": rep["err_inf"],
                     "err_mean_abs": rep["err_mean_abs"], "reached": bool(rep["err_met"])}
        finals[name] = u
    if out["fp64"]["reached"] and out["fp32_refine"]["reached"]:
        out["speedup_fp32_refine"] = round(out["fp64"]["wall_s"] / out["fp32_refine"]["wall_s"], 3)
    if out["fp64"]["steps"] == out["fp32_refine"]["steps"]:
        # the two final iterates after the same number of steps
        out["max_abs_diff_fp32_refine_vs_fp64"] = (finals["fp32_refine"] - finals["fp64"]).abs().max().item()
    return out


def run_cube1m_fp32(steps=2000, warmup=500, inner=500):
    """FP32 inner sweeps of the mixed mode on cube1M, m = 4: outer passes of
    `inner` FP32 steps, each after one FP64 residual.  Device time per inner
    step (the outer residuals included: one per `inner` steps) and the stream
    rates against 8n + 12 algorithmic bytes and against the bytes as stored."""
    from paper_2502_12878_amd import RBF_MODE_MIXED
    s = setup_problem(4, keep_fp32=True)
    p, wl = s["p"], s["wl"]
    nint = int((s["typ"] == 0).sum())
    u = s["u0"].clone()
    st, _ = p.iterate(s["f"], u, wl.dt, warmup, 0.0, inner, mode=RBF_MODE_MIXED, inner_steps=inner)
    assert st == 0, st
    u = s["u0"].clone()
    st, rep = p.iterate(s["f"], u, wl.dt, steps, 0.0, inner, mode=RBF_MODE_MIXED, inner_steps=inner)
    assert st == 0 and rep["steps"] == steps, (st, rep)
    per = rep["seconds"] / rep["steps"]
    info = p.operator_info()
    alg = (8 * wl.n + 12) * nint
    out = {"workload": f"cube1M_fp32: 3D 100^3 jittered grid (seed 1), m=4, n={wl.n}, FP32 inner sweeps of {inner} "
                       f"steps inside the FP64 residual correction",
           "steps": rep["steps"], "device_s": round(rep["seconds"], 4), "ms_per_inner_step": 1e3 * per,
           "node_updates_per_s": nint / per, "alg_bytes_per_update": 8 * wl.n + 12, "alg_GBps": alg / per / 1e9,
           "hbm_frac": alg / per / 1e9 / PEAK_HBM_GBS, "format_bytes_per_sweep": info["stream_bytes_f32"],
           "format_GBps": info["stream_bytes_f32"] / per / 1e9,
           "sweep_shape": {k[4:]: v for k, v in info.items() if k.startswith("f32_")}}
    p.close()
    return out


def _time_oracle_sweeps(op, f, u0, dt, threads, budget_s, min_sweeps):
    """Node-update rate of the oracle's OpenMP sweep (row-parallel for) with
    `threads` threads: at least `min_sweeps` sweeps and `budget_s` seconds,
    after one untimed sweep."""
    a, b = u0.copy(), u0.copy()
    op.sweep_omp(f, dt, a, b, threads)
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        op.sweep_omp(f, dt, a, b, threads)
        a, b = b, a
        sweeps += 1
        el = time.perf_counter() - t0
        if sweeps >= min_sweeps and el >= budget_s:
            return sweeps, el


def cpu_baseline(s, budget_s=8.0):
    """The oracle's OpenMP sweep (the paper's intra-node row-parallel loop)
    on the headline operator itself: the supports and weights of the 1M-node
    cube exported from the library (rbf_get_stencils / rbf_get_weights),
    timed with every host core the process may use and with one thread.  A
    30^3 instance of the same workload, whose operator the oracle builds
    itself, is timed beside it as a secondary figure."""
    import numpy as np

    import oracle
    import rbf_inputs as ri
    threads = len(os.sched_getaffinity(0))
    p = s["p"]
    typ = s["typ"]
    nint = int((typ == 0).sum())
    op = oracle.Operator(typ, p.get_stencils(), p.get_weights())
    f, u0, dt = s["f_h"], s["u0_h"], s["wl"].dt
    sw_all, el_all = _time_oracle_sweeps(op, f, u0, dt, threads, budget_s, 20)
    sw_one, el_one = _time_oracle_sweeps(op, f, u0, dt, 1, budget_s / 2, 2)
    del op
    # secondary: 30^3 instance built by the oracle
    side, m, n = 30, 4, 70
    xyz3, typ3 = ri.jittered_grid(3, side, 0.3, 1)
    idx3, w3 = oracle.setup(xyz3, typ3, n, m=m)
    _, f3, _, u03 = ri.manufactured(3, xyz3, typ3)
    op3 = oracle.Operator(typ3, idx3, w3)
    nint3 = int((typ3 == 0).sum())
    h3 = ri.grid_spacing(side)
    sw3, el3 = _time_oracle_sweeps(op3, f3, u03, 0.15 * h3 * h3 / 6, threads, 2.0, 20)
    return {"value": nint * sw_all / el_all, "unit": "node-updates/s", "cores": threads, "kind": "oracle",
            "single_thread_value": nint * sw_one / el_one,
            "sweeps_timed": sw_all, "single_thread_sweeps_timed": sw_one,
            "alg_GBps": round((12 * 70 + 24) * nint * sw_all / el_all / 1e9, 2),
            "sample": f"oracle OpenMP sweep (row-parallel for) on the cube1M m=4 operator exported from the GPU "
                      f"({nint} interior rows, n=70): {sw_all} sweeps on {threads} threads ({el_all:.1f} s) and "
                      f"{sw_one} on 1 thread ({el_one:.1f} s), after one untimed sweep each",
            "secondary_30cube": {"value": nint3 * sw3 / el3, "interior_nodes": nint3, "sweeps_timed": sw3,
                                 "note": "same generator and parameters at 30^3 (operator built by the oracle; "
                                         "~19 MB, partly cache-resident on the host)"}}


def run_c2_block(steps=2000, warmup=1000, inner=500, target=1e-6, builder_steps_to_target=740_500):
    """The 8M-node cube (200^3, seed 2, m = 4, n = 70): `steps` explicit steps
    in each mode, plain FP64 sweeps and FP32 inner sweeps of `inner` steps
    inside the FP64 residual correction, with the error against the exact
    solution checked every 500 steps as in a time-to-error run; device and
    wall time per step, their ratio, and both iterates compared.  Time to
    L-inf error `target` is extrapolated from the step count the full runs
    needed (measured by the builder, 740,500 steps in both modes)."""
    import torch

    import rbf_inputs as ri
    from paper_2502_12878_amd import RBF_MODE_FP64, RBF_MODE_MIXED, Problem
    wl = ri.workload("cube8M")
    p = Problem(0)
    t0 = time.perf_counter()
    xd, td = p.build_nodes(wl.dim, wl.side, wl.jitter, wl.seed)
    p.set_nodes(xd, td)
    del xd, td
    p.build_stencils(wl.n)
    p.compute_weights(wl.m, keep_fp32=True)
    p.autotune()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    xyz_h, typ_h = wl.nodes()
    u_ex, f, g, u0 = ri.manufactured(wl.dim, xyz_h, typ_h)
    nint = int((typ_h == 0).sum())
    del xyz_h
    fd, uref, u0d = _dev(f), _dev(u_ex), _dev(u0)
    del u_ex, f, g
    out = {"workload": f"cube8M: 3D 200^3 jittered grid (seed 2), m=4, n=70, dt=0.15*h^2/6, {steps} steps per mode "
                       f"(error vs exact checked every 500 steps)", "interior_nodes": nint,
           "setup_s": round(setup_s, 2)}
    finals = {}
    for name, mode in (("fp64", RBF_MODE_FP64), ("fp32_refine", RBF_MODE_MIXED)):
        kw = dict(mode=mode, inner_steps=inner, u_ref=uref, err_target=target)
        u = u0d.clone()
        p.iterate(fd, u, wl.dt, warmup, 0.0, 500, **kw)  # builds the graphs the timed call uses
        u = u0d.clone()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, rep = p.iterate(fd, u, wl.dt, steps, 0.0, 500, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        assert rep["steps"] == steps, rep
        per = rep["seconds"] / steps
        alg = (12 * wl.n + 24) if mode == RBF_MODE_FP64 else (8 * wl.n + 12)
        out[name] = {"status": st, "steps": steps, "device_s": round(rep["seconds"], 4), "wall_s": round(wall, 4),
                     "ms_per_step_device": round(1e3 * per, 5), "ms_per_step_wall": round(1e3 * wall / steps, 5),
                     "alg_bytes_per_update": alg, "alg_GBps": round(alg * nint / per / 1e9, 1),
                     "err_inf_vs_exact": rep["err_inf"],
                     "time_to_error_extrapolated_s": round(per * builder_steps_to_target, 1)}
        finals[name] = u
        _progress(f"cube8M {name}: {1e3 * per:.4f} ms per step (device), err_inf {rep['err_inf']:.3e}")
    corr = (finals["fp64"] - u0d).abs().max().item()
    out["max_abs_diff_fp32_refine_vs_fp64"] = (finals["fp32_refine"] - finals["fp64"]).abs().max().item()
    out["correction_max_abs"] = corr
    out["speedup_fp32_refine_device"] = round(out["fp64"]["ms_per_step_device"] /
                                              out["fp32_refine"]["ms_per_step_device"], 3)
    out["speedup_fp32_refine_wall"] = round(out["fp64"]["ms_per_step_wall"] / out["fp32_refine"]["ms_per_step_wall"], 3)
    out["steps_to_target"] = {"value": builder_steps_to_target, "target_err_inf": target,
                              "source": "measured by the builder in full runs of both modes to the target "
                                        "(bench.py --workload cube8M --mode fp64 / fp32_refine); not re-run here"}
    p.close()
    del finals, fd, uref, u0d
    torch.cuda.empty_cache()
    return out


def _progress(msg):
    print(msg, file=sys.stderr, flush=True)


def _dev(a):
    import torch
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def run_cube8m(mode_name, target, piece_steps=40000, max_steps=3_000_000, cpu_sweeps=3):
    """Time to L-inf error `target` against the exact solution on the 8M-node
    cube (m = 4, n = 70), FP64 or FP32 inner sweeps with FP64 refinement; the
    error is checked every 500 steps in both modes.  Runs in pieces of
    `piece_steps` steps (the state is just u) so progress is printed.  In FP64
    mode the oracle's OpenMP sweep is then timed on the same operator (copied
    to the host) for `cpu_sweeps` steps, and the CPU time to the target is
    extrapolated as the GPU's step count times that time per step."""
    import torch

    import rbf_inputs as ri
    from paper_2502_12878_amd import RBF_MODE_FP64, RBF_MODE_MIXED, Problem
    mode = RBF_MODE_MIXED if mode_name == "fp32_refine" else RBF_MODE_FP64
    wl = ri.workload("cube8M")
    p = Problem(0)
    t0 = time.perf_counter()
    xyz, typ = p.build_nodes(wl.dim, wl.side, wl.jitter, wl.seed)
    p.set_nodes(xyz, typ)
    del xyz, typ
    p.build_stencils(wl.n)
    p.compute_weights(wl.m, keep_fp32=(mode == RBF_MODE_MIXED))
    p.autotune()
    setup_s = time.perf_counter() - t0
    xyz_h, typ_h = wl.nodes()
    u_ex, f, g, u0 = ri.manufactured(wl.dim, xyz_h, typ_h)
    nint = int((typ_h == 0).sum())
    del xyz_h
    fd, uref, u = _dev(f), _dev(u_ex), _dev(u0)
    steps = 0
    dev_s = 0.0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    rep = None
    while steps < max_steps:
        st, rep = p.iterate(fd, u, wl.dt, piece_steps, 0.0, 500, mode=mode, inner_steps=500, u_ref=uref,
                            err_target=target)
        steps += rep["steps"]
        dev_s += rep["seconds"]
        _progress(f"cube8M {mode_name}: {steps} steps, err_inf {rep['err_inf']:.3e}, device {dev_s:.1f} s")
        # a piece that ends before the target reports "not converged" (5); go on
        if rep["err_met"] or st not in (0, 5):
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    sample = u[:: 1009].cpu().numpy()
    cpu = None
    if mode == RBF_MODE_FP64 and cpu_sweeps > 0:
        import oracle
        _progress("cube8M: timing the oracle's OpenMP sweep on the same operator")
        op = oracle.Operator(typ_h, p.get_stencils(), p.get_weights())
        threads = len(os.sched_getaffinity(0))
        a, b = u0.copy(), u0.copy()
        op.sweep_omp(f, wl.dt, a, b, threads)  # untimed first sweep
        t1 = time.perf_counter()
        for _ in range(cpu_sweeps):
            op.sweep_omp(f, wl.dt, a, b, threads)
            a, b = b, a
        s_step = (time.perf_counter() - t1) / cpu_sweeps
        cpu = {"kind": "extrapolated", "threads": threads, "sweeps_timed": cpu_sweeps, "oracle_s_per_step": s_step,
               "node_updates_per_s": nint / s_step, "time_to_error_s": round(s_step * steps, 1),
               "how": "the GPU's steps to the target times the oracle's OpenMP sweep time per step on the same "
                      "operator"}
        del op
    return {"workload": "cube8M: 3D 200^3 jittered grid (seed 2), m=4, n=70, dt=0.15*h^2/6", "mode": mode_name,
            "cpu_time_to_error": cpu,
            "target_err_inf": target, "reached": bool(rep["err_met"]), "steps": steps, "wall_s": round(wall, 2),
            "device_s": round(dev_s, 2), "ms_per_step": 1e3 * dev_s / max(1, steps), "err_inf": rep["err_inf"],
            "err_mean_abs": rep["err_mean_abs"], "interior_nodes": nint, "setup_s": round(setup_s, 2),
            "alg_bytes_per_update": 12 * wl.n + 24 if mode == RBF_MODE_FP64 else 8 * wl.n + 12,
            "u_sample_every_1009": {"sum": float(sample.sum()), "sumsq": float((sample ** 2).sum())}}


def ns_flops(n, M):
    """FP64 flops of the null-space weight solver's steps for one system of n
    support nodes and M monomials (K = n - M): the LU of P with the extra
    right-hand-side row, the K + 1 triangular solves for [X v1], the block
    products T = A [G v] (pivot columns only) and C_aug = [G v]^T T (lower
    triangle), the Cholesky of C with the reduced right-hand side as an
    extra row, the backward substitution and w = v + G z.  Work the kernels
    also do on tile padding and on the upper halves of diagonal tiles is not
    counted."""
    K = n - M
    lu = sum(2 * (n - k) * (M - k - 1) for k in range(M))
    xs = (K + 1) * M * (M - 1)
    gemm = 2 * n * M * (K + 1) + M * (K + 1) * (K + 2)
    chol = sum(2 * (K - k) * (K - k + 1) // 2 for k in range(K)) + 2 * sum(K - k - 1 for k in range(K))
    return lu + xs + gemm + chol + K * K + 2 * M * K


def gepp_flops(S):
    """Flops of Gaussian elimination with back substitution on S unknowns
    (one right-hand side): the elimination-equivalent count."""
    return sum(2.0 * (S - k - 1) * (S - k) for k in range(S)) + 2.0 * S * S


def run_cube4m_bands(steps=1000):
    """Per-node orders by distance to the boundary (m = 2 / 4 / 6, n = 20 / 70 /
    168) on the 159^3 cube: supports with per-node sizes, every weight system in
    one persistent launch per solver size, then FP64 sweeps on the sliced
    operator.  Systems above 40 unknowns go to the null-space solver (the
    others to the one-wavefront elimination); the roofline counts the flops
    that solver executes, against the FP64 peak."""
    import numpy as np
    import torch

    import rbf_inputs as ri
    from paper_2502_12878_amd import Problem
    wl = ri.workload("cube4M_bands")
    xyz_h, typ_h = wl.nodes()
    m, n = ri.order_bands(3, xyz_h, typ_h, wl.h)
    interior = typ_h == 0
    classes = {}
    flops_equiv = 0.0
    flops_exec = 0.0
    alg_bytes = 0
    for mm in (2, 4, 6):
        sel = interior & (m == mm)
        cnt = int(sel.sum())
        nn = 2 * ri.num_monomials(3, mm)
        M = ri.num_monomials(3, mm)
        S = nn + M
        ns = S > 40
        classes[str(mm)] = {"rows": cnt, "n": nn, "S": S, "solver": "null-space" if ns else "elimination"}
        flops_equiv += cnt * gepp_flops(S)
        flops_exec += cnt * (ns_flops(nn, M) if ns else gepp_flops(S))
        alg_bytes += cnt * (12 * nn + 24)
    p = Problem(0)
    xd, td = p.build_nodes(3, wl.side, wl.jitter, wl.seed)
    p.set_nodes(xd, td)
    del xd, td
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.build_stencils(n_per_node=n)
    t1 = time.perf_counter()
    p.compute_weights(m_per_node=m)
    t2 = time.perf_counter()
    info = p.operator_info()
    p.autotune()
    u_ex, f, g, u0 = ri.manufactured(3, xyz_h, typ_h)
    s = {"p": p, "wl": wl, "f": _dev(f), "u0": _dev(u0)}
    wall, per_sweep, nsw, rep, _ = time_sweeps(s, steps, 100)
    nint = int(interior.sum())
    tw = t2 - t1
    return {"workload": "cube4M_bands: 3D 159^3 jittered grid (seed 3), m=2/4/6 by distance to the boundary "
                        "(<3h, <6h, else), n=2M", "classes": classes, "interior_nodes": nint,
            "ns_systems": info["ns_systems"], "elim_systems": info["elim_systems"],
            "stencils_s": round(t1 - t0, 3), "weights_s": round(tw, 3),
            # elimination-equivalent rate (the flops Gaussian elimination would
            # take for the same systems), comparable across solvers
            "weights_gflops": round(flops_equiv / tw / 1e9, 1), "weights_flop_total": flops_equiv,
            "weights_flop_executed": flops_exec,
            "weights_roofline": {"bound": "fp64 (matrix cores and FMA); LDS and the pivot chains in practice",
                                 "achieved": round(flops_exec / tw / 1e12, 3), "peak": PEAK_FP64_FLOPS / 1e12,
                                 "unit": "TFLOP/s", "frac": round(flops_exec / tw / PEAK_FP64_FLOPS, 4)},
            "sweep_kernel_ms": round(1e3 * per_sweep, 4), "node_updates_per_s": nint / per_sweep,
            "sweep_alg_GBps": round(alg_bytes / per_sweep / 1e9, 1),
            "sweep_hbm_frac": round(alg_bytes / per_sweep / 1e9 / PEAK_HBM_GBS, 4), "res_final": rep["res_final"]}


def run_cube2m_adjoint(directions=32, cpu_K=20):
    """dJ/df for J = 1/2 |u_K - u_target|^2 (interior) after K = 2000 steps on
    the 126^3 cube (m = 4), by checkpointed forward + transposed sweeps, against
    central differences on `directions` seeded smooth directions; and the
    gradient of the first `cpu_K` steps against the oracle's sequential
    transposed loop on the same 2M-node operator (the CPU reference gradient;
    the full K would take the sequential oracle tens of minutes)."""
    import numpy as np
    import torch

    import oracle
    import rbf_inputs as ri
    from paper_2502_12878_amd import Problem, SolveK
    wl = ri.workload("cube2M_adjoint")
    K, every = wl.extra["K"], wl.extra["every"]
    p = Problem(0)
    xd, td = p.build_nodes(3, wl.side, wl.jitter, wl.seed)
    p.set_nodes(xd, td)
    del xd, td
    p.build_stencils(wl.n)
    p.compute_weights(wl.m)
    p.autotune()
    xyz_h, typ_h = wl.nodes()
    I = typ_h == 0
    It = torch.tensor(I, device="cuda")
    f = _dev(np.where(I, ri.gaussian_field(3, xyz_h, wl.seed + 100), 0.0))
    f_t = f + 0.1 * _dev(np.where(I, ri.gaussian_field(3, xyz_h, wl.seed + 200), 0.0))
    zero = torch.zeros_like(f)
    with torch.no_grad():
        u_t = SolveK.apply(f_t, p, zero, K, every, wl.dt)

    def J(ff):
        d = (SolveK.apply(ff, p, zero, K, every, wl.dt) - u_t)[It]
        return 0.5 * (d * d).sum()

    # first backward: builds the transposed operator and its codes and picks
    # the transposed sweep's shape (timed separately); then the timed pass
    fr = f.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J(fr).backward()
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    fr = f.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = J(fr)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    grad = fr.grad.detach()
    eps = 1e-2 * f.abs().max().item()
    gnorm = grad.norm().item()
    errs = []
    with torch.no_grad():
        j = 0
        seed_off = 0
        while len(errs) < directions:
            v = _dev(np.where(I, ri.gaussian_field(3, xyz_h, wl.seed + 300 + j + seed_off), 0.0))
            v = v / v.abs().max()
            fd = ((J(f + eps * v) - J(f - eps * v)) / (2 * eps)).item()
            if abs(fd) < 1e-3 * gnorm * v.norm().item():
                seed_off += 1000  # deterministic redraw of a direction nearly orthogonal to the gradient
                continue
            errs.append(abs((grad * v).sum().item() - fd) / abs(fd))
            _progress(f"direction {j}: rel err {errs[-1]:.2e}")
            j += 1
        # CPU reference gradient: dJ/du_K of this problem, cpu_K transposed
        # steps on the library's operator, GPU vs the oracle's loop
        gK = torch.where(It, SolveK.apply(f, p, zero, K, every, wl.dt) - u_t, zero)
    sten = p.get_stencils()
    op = oracle.Operator(typ_h, sten, p.get_weights())
    gK_h = gK.cpu().numpy()
    g_gpu = p.adjoint_f(gK, cpu_K, cpu_K, wl.dt).cpu().numpy()
    t3 = time.perf_counter()
    g_cpu = op.adjoint_f(wl.dt, cpu_K, gK_h)
    cpu_s = time.perf_counter() - t3
    cpu_rel = float(np.abs(g_gpu - g_cpu).max() / np.abs(g_cpu).max())
    _progress(f"CPU reference gradient ({cpu_K} steps): rel diff {cpu_rel:.2e}, oracle {cpu_s:.1f} s")
    del op
    # algorithmic bytes per step: forward 12n + 24 per interior row; a
    # transposed step (Horner form: the forward sweep on L_II^T) 12 B per
    # entry of L_II plus f, T and T_new (24 B) per interior row
    valid = sten[I] >= 0
    nnz = int((valid & (typ_h[np.where(valid, sten[I], 0)] == 0)).sum())
    del sten, valid
    nint = int(I.sum())
    fwd_bytes = (12 * wl.n + 24) * nint
    adj_bytes = 12 * nnz + 24 * nint
    fwd_ms, adj_ms = 1e3 * (t1 - t0) / K, 1e3 * (t2 - t1) / K
    info = p.operator_info()
    p.close()
    return {"workload": "cube2M_adjoint: 3D 126^3 jittered grid (seed 4), m=4, n=70, K=2000, checkpoints every 100",
            "interior_nodes": nint, "nnz_L_II": nnz, "forward_alg_GBps": round(fwd_bytes / fwd_ms / 1e6, 1),
            "adjoint_alg_GBps": round(adj_bytes / adj_ms / 1e6, 1),
            "adjoint_hbm_frac": round(adj_bytes / adj_ms / 1e6 / PEAK_HBM_GBS, 4),
            "forward_ckpt_s": round(t1 - t0, 3), "adjoint_s": round(t2 - t1, 3),
            "first_forward_and_adjoint_s": round(first_s, 3),
            "adjoint_ms_per_step": round(1e3 * (t2 - t1) / K, 4), "forward_ms_per_step": round(1e3 * (t1 - t0) / K, 4),
            "transposed_operator": {k: info[k] for k in ("t_slices", "t_slots", "t_coded_slices", "t_code_mismatches",
                                                         "t_max_len", "t_waves", "t_unroll", "t_codes",
                                                         "t_lane_order", "t_masked")},
            "J": loss.item(), "fd_eps": eps, "directions": directions, "max_rel_err_vs_fd": max(errs),
            "median_rel_err_vs_fd": float(np.median(errs)), "rel_errs": errs,
            "cpu_reference_gradient": {"steps": cpu_K, "rel_diff_gpu_vs_oracle": cpu_rel, "oracle_s": round(cpu_s, 2),
                                       "how": "dJ/du_K of the K=2000 problem pulled back through the first "
                                              f"{cpu_K} transposed steps by the library and by the oracle's "
                                              "sequential scatter loop on the library's operator"}}


def run_support_sweep(m=2, sizes=(20, 30, 40, 60, 80, 100, 130, 168), steps=1000):
    """Support size beyond 2M at fixed order (the compute-time model t ~ n of
    the paper's support-size study): sweep time, node-updates/s and algorithmic
    GB/s per n on the 1M-node cube, plus the truncation error
    max |L_h u_exact - f| of each operator."""
    import numpy as np
    import torch

    import rbf_inputs as ri
    from paper_2502_12878_amd import Problem
    wl = ri.workload("cube1M", m=m)
    xyz_h, typ_h = wl.nodes()
    u_ex, f, g, u0 = ri.manufactured(3, xyz_h, typ_h)
    nint = int((typ_h == 0).sum())
    rows = []
    for n in sizes:
        p = Problem(0)
        xd, td = p.build_nodes(3, wl.side, wl.jitter, wl.seed)
        p.set_nodes(xd, td)
        del xd, td
        t0 = time.perf_counter()
        p.build_stencils(n)
        p.compute_weights(m)
        setup = time.perf_counter() - t0
        p.autotune()
        s = {"p": p, "wl": wl, "f": _dev(f), "u0": _dev(u0)}
        wall, per_sweep, nsw, rep, _ = time_sweeps(s, steps, 100)
        trunc = p.residual(s["f"], _dev(u_ex))
        rows.append({"n": n, "setup_s": round(setup, 3), "kernel_ms_per_sweep": round(1e3 * per_sweep, 4),
                     "node_updates_per_s": nint / per_sweep,
                     "alg_GBps": round(nint * (12 * n + 24) / per_sweep / 1e9, 1), "truncation_err_inf": trunc})
        _progress(f"n={n}: {1e3 * per_sweep:.4f} ms per sweep, truncation {trunc:.3e}")
        p.close()
    ns = np.array([r["n"] for r in rows], dtype=float)
    ts = np.array([r["kernel_ms_per_sweep"] for r in rows])
    slope = float(np.polyfit(np.log(ns), np.log(ts), 1)[0])
    a, b = np.polyfit(12 * ns + 24, ts, 1)
    return {"workload": f"cube1M support sweep: 3D 100^3 jittered grid (seed 1), m={m}, n in {list(sizes)}",
            "interior_nodes": nint, "rows": rows, "loglog_slope_t_vs_n": round(slope, 3),
            "fit_ms_per_byte_per_row": a, "fit_ms_offset": b}


def run_square10k(chunks=(100, 1000, 5000)):
    """The 2D 10k-node case (100^2 jittered grid, seed 0, m = 2, n = 12), a
    cache- and launch-bound problem rather than a bandwidth point.  At the
    literal step 0.9 dt_max the iteration diverges: the step where the GPU
    and the oracle stop is reported.  At 0.15 dt_max, 20,000 steps run on the
    GPU (graph chunks of several lengths, each graph built before timing) and
    for real in the oracle's sequential sweep; errors against the exact
    solution (L-inf and the mean absolute error over all nodes) and the
    GPU-oracle difference are reported."""
    import numpy as np
    import torch

    import oracle
    import rbf_inputs as ri
    from paper_2502_12878_amd import Problem
    out = {"workload": "square10k: 2D 100^2 jittered grid (seed 0), m=2, n=12, 20,000 steps"}
    for name in ("square10k", "square10k_stable"):
        wl = ri.workload(name)
        xyz, typ = wl.nodes()
        u_ex, f, g, u0 = ri.manufactured(2, xyz, typ)
        steps = wl.extra["steps"]
        p = Problem(0)
        xd, td = p.build_nodes(2, wl.side, wl.jitter, wl.seed)
        p.set_nodes(xd, td)
        p.build_stencils(wl.n)
        p.compute_weights(wl.m)
        p.autotune()
        fd, uref = _dev(f), _dev(u_ex)
        idx, w = oracle.setup(xyz, typ, wl.n, m=wl.m)
        op = oracle.Operator(typ, idx, w)
        t0 = time.perf_counter()
        uo, rep_o, st_o = op.iterate(f, wl.dt, u0, steps, 0.0, 1000)
        cpu_s = time.perf_counter() - t0
        if name == "square10k":
            u = _dev(u0)
            st, rep = p.iterate(fd, u, wl.dt, steps, 0.0, 1000, u_ref=uref)
            out["literal_0.9dt_max"] = {"status": st, "diverged_step": rep["diverged_step"],
                                        "oracle_status": st_o, "oracle_diverged_step": rep_o["diverged_step"]}
            p.close()
            continue
        runs = []
        for chunk in chunks:
            u = _dev(u0)
            p.iterate(fd, u, wl.dt, chunk, 0.0, chunk, u_ref=uref)  # builds the chunk's graph
            u = _dev(u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, rep = p.iterate(fd, u, wl.dt, steps, 0.0, chunk, u_ref=uref)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            runs.append({"chunk": chunk, "status": st, "wall_s": round(wall, 4),
                         "us_per_step": round(1e6 * wall / steps, 3), "steps_per_s": round(steps / wall, 1)})
            _progress(f"square10k chunk {chunk}: {1e6 * wall / steps:.3f} us per step")
        ug = u.cpu().numpy()
        nint = int((typ == 0).sum())
        best = min(r["wall_s"] for r in runs)
        out["stable_0.15dt_max"] = {
            "interior_nodes": nint, "runs": runs, "best_steps_per_s": round(steps / best, 1),
            "best_node_updates_per_s": nint * steps / best, "err_inf": rep["err_inf"],
            "err_mean_abs": rep["err_mean_abs"], "rel_diff_vs_oracle": float(np.abs(ug - uo).max() / np.abs(uo).max()),
            "oracle_sequential_s": round(cpu_s, 3), "oracle_steps_per_s": round(steps / cpu_s, 1)}
        p.close()
    return out


def _converge(p, fd, u, dt, uref, tol_rel, max_steps, chunk=500, stall=10):
    """Iterate to relative residual `tol_rel` (or a 10-chunk stall at the
    rounding floor); returns the report with the final errors."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rep = p.iterate(fd, u, dt, max_steps, tol_rel, chunk, stall_chunks=stall, u_ref=uref)
    torch.cuda.synchronize()
    rep["wall_s"] = time.perf_counter() - t0
    rep["status"] = st
    return rep


def run_order_scan(orders=(2, 4, 6), sides=(21, 31, 46, 68, 100), alpha=0.15, tol_rel=1e-11, seed=1):
    """Augmentation order x node spacing (the paper's time/error scan, Sec.
    III-B): for each (m, h) on the 3D jittered cube, the wall time per step
    t_ws, the derived t_T / T = t_ws / (alpha dt_max) with dt_max = h^2/(2d),
    the steps and wall time to converge, and the error of the converged
    solution against the exact one (mean |u - u_a| over all nodes as in the
    paper, and L-inf)."""
    import numpy as np

    import rbf_inputs as ri
    from paper_2502_12878_amd import Problem
    rows = []
    for m in orders:
        n = 2 * ri.num_monomials(3, m)
        for side in sides:
            h = ri.grid_spacing(side)
            dt_max = h * h / 6
            dt = alpha * dt_max
            xyz_h, typ_h = ri.jittered_grid(3, side, 0.3, seed)
            u_ex, f, g, u0 = ri.manufactured(3, xyz_h, typ_h)
            nint = int((typ_h == 0).sum())
            p = Problem(0)
            xd, td = p.build_nodes(3, side, 0.3, seed)
            p.set_nodes(xd, td)
            del xd, td
            t0 = time.perf_counter()
            p.build_stencils(n)
            p.compute_weights(m)
            setup = time.perf_counter() - t0
            if nint >= 200_000:
                p.autotune()
            fd, uref = _dev(f), _dev(u_ex)
            # step time: 2000 steps in graph chunks of 500, after 500 warm-up steps
            u = _dev(u0)
            p.iterate(fd, u, dt, 500, 0.0, 500)
            u = _dev(u0)
            torch_sync()
            t1 = time.perf_counter()
            st, rep = p.iterate(fd, u, dt, 2000, 0.0, 500)
            torch_sync()
            t_ws = (time.perf_counter() - t1) / 2000
            per_sweep, _ = p.last_sweep_time()
            u = _dev(u0)
            rc = _converge(p, fd, u, dt, uref, tol_rel, max_steps=int(60.0 / (alpha * h * h)) + 1000)
            rows.append({"m": m, "n": n, "side": side, "h": h, "interior_nodes": nint, "setup_s": round(setup, 3),
                         "t_ws_ms": 1e3 * t_ws, "kernel_ms_per_sweep": 1e3 * per_sweep,
                         "tT_over_T_s": t_ws / (alpha * dt_max), "steps_to_converge": rc["steps"],
                         "converged": bool(rc["converged"]), "res_final_rel": rc["res_final"] / rc["fnorm"],
                         "time_to_converge_s": round(rc["wall_s"], 3), "err_mean_abs": rc["err_mean_abs"],
                         "err_inf": rc["err_inf"]})
            _progress(f"scan m={m} side={side}: t_ws {1e3 * t_ws:.4f} ms, {rc['steps']} steps, "
                      f"err_inf {rc['err_inf']:.3e}, mean {rc['err_mean_abs']:.3e}")
            p.close()
    slopes = {}
    for m in orders:
        r = [x for x in rows if x["m"] == m and x["converged"]]
        if len(r) >= 3:
            slopes[str(m)] = round(float(np.polyfit(np.log([x["h"] for x in r]),
                                                    np.log([x["err_inf"] for x in r]), 1)[0]), 3)
    return {"workload": f"order x spacing scan: 3D jittered cube (seed {seed}), m in {list(orders)}, "
                        f"side in {list(sides)}, n = 2M, dt = {alpha}*h^2/6, converged to relative residual "
                        f"{tol_rel} (or a stall at the rounding floor)",
            "rows": rows, "err_inf_slope_vs_h": slopes}


def run_mixed_bc(side=100, m=4, steps=3000, conv_sides=(21, 31, 46), conv_orders=(2, 4), alpha=0.15, seed=5):
    """The mixed Dirichlet/Neumann variant on [0, 1/2]^3: sweep throughput with
    the Neumann update before every step on the side^3 grid, and the error of
    the converged solution under refinement at small sizes."""
    import numpy as np

    import rbf_inputs as ri
    from paper_2502_12878_amd import Problem

    def build(sd, mm):
        xyz, typ, normals = ri.mixed_bc_grid(3, sd, 0.3, seed)
        u_ex, f, u0 = ri.manufactured_mixed(3, xyz, typ)
        p = Problem(0)
        p.set_nodes(xyz, typ)
        p.set_normals(normals)
        t0 = time.perf_counter()
        p.build_stencils(2 * ri.num_monomials(3, mm))
        p.compute_weights(mm)
        return p, typ, u_ex, f, u0, time.perf_counter() - t0

    p, typ, u_ex, f, u0, setup = build(side, m)
    p.autotune()
    h = 0.5 / (side - 1)
    dt = alpha * h * h / 6
    nint, nneu = int((typ == 0).sum()), int((typ == 2).sum())
    fd = _dev(f)
    u = _dev(u0)
    p.iterate(fd, u, dt, 500, 0.0, 500)
    u = _dev(u0)
    torch_sync()
    t0 = time.perf_counter()
    st, rep = p.iterate(fd, u, dt, steps, 0.0, 500)
    torch_sync()
    wall = time.perf_counter() - t0
    per_step, nsw = p.last_sweep_time()
    n = 2 * ri.num_monomials(3, m)
    p.close()
    _progress(f"mixed_bc side={side}: {1e3 * per_step:.4f} ms per step (sweep + Neumann update)")
    conv = []
    for mm in conv_orders:
        for sd in conv_sides:
            q, typ2, ue, f2, u02, _ = build(sd, mm)
            hh = 0.5 / (sd - 1)
            rc = _converge(q, _dev(f2), _dev(u02), alpha * hh * hh / 6, _dev(ue), 1e-11,
                           max_steps=int(30.0 / (alpha * hh * hh)) + 1000)
            conv.append({"m": mm, "side": sd, "h": hh, "steps": rc["steps"], "converged": bool(rc["converged"]),
                         "err_inf": rc["err_inf"], "err_mean_abs": rc["err_mean_abs"]})
            _progress(f"mixed_bc m={mm} side={sd}: {rc['steps']} steps, err_inf {rc['err_inf']:.3e}")
            q.close()
    slopes = {}
    for mm in conv_orders:
        r = [x for x in conv if x["m"] == mm]
        if len(r) >= 2:
            slopes[str(mm)] = round(float(np.polyfit(np.log([x["h"] for x in r]),
                                                     np.log([x["err_inf"] for x in r]), 1)[0]), 3)
    return {"workload": f"mixed_bc: [0,1/2]^3, {side}^3 jittered grid (seed {seed}), Dirichlet on the outer faces, "
                        f"zero normal derivative on the inner faces, m={m}, n={n}, dt={alpha}*h^2/6",
            "interior_nodes": nint, "neumann_nodes": nneu, "setup_s": round(setup, 3),
            "ms_per_step_device": 1e3 * per_step, "ms_per_step_wall": 1e3 * wall / steps,
            "node_updates_per_s": nint / per_step,
            "alg_GBps_interior_sweep": round(nint * (12 * n + 24) / per_step / 1e9, 1),
            "convergence": conv, "err_inf_slope_vs_h": slopes}


def torch_sync():
    import torch
    torch.cuda.synchronize()


def stream_ceiling(nbytes=1 << 30, reps=20):
    """Achievable HBM rates on this device for context: a 1 GiB device copy
    (read + write) and a 1 GiB read-only sum, timed with events."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    out = {}
    for name, fn, moved in (("copy", lambda: y.copy_(x), 2 * nbytes), ("read", lambda: x.sum(), nbytes)):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[f"{name}_GBps"] = round(moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del x, y
    torch.cuda.empty_cache()
    return out


def calibrate_copy(nbytes=1 << 30, reps=10):
    """A plain device copy of known size, for scaling rocprofv3 FETCH_SIZE /
    WRITE_SIZE readings to bytes."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes,
                      "launches": reps}))


def _counter_per_dispatch(csv_dir, match, largest=False):
    """Mean counter value (KiB) per dispatch of the most often dispatched
    kernel whose name contains `match` (the timed launches), from a rocprofv3
    --pmc csv output directory (one counter per run); its name and dispatch
    count too."""
    import csv
    import glob
    vals = {}
    for path in glob.glob(os.path.join(csv_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if match in r["Kernel_Name"]:
                    per = vals.setdefault(r["Kernel_Name"], {})
                    d = (path, r["Dispatch_Id"])
                    per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
    if not vals:
        raise SystemExit(f"no dispatch of {match!r} under {csv_dir}")
    name, per = max(vals.items(), key=lambda kv: len(kv[1]))
    v = list(per.values())
    if largest:  # only the big launches (the calibration copies, not incidental small ones)
        v = [x for x in v if x >= 0.5 * max(v)]
    return sum(v) / len(v), len(v), name


def record_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, bench_json):
    """Write the HBM traffic of the timed FP64 sweep into profiles/traffic.json
    from four rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE of the bench
    line, then of `--calibrate-copy`) and the bench line those runs printed
    (for the sweep shape and the algorithmic bytes)."""
    with open(bench_json) as fh:
        line = json.loads(fh.read().strip().splitlines()[-1])
    rf = line["roofline"]
    sh = rf["sweep_shape"]
    shape = ",".join(str(sh[k]) for k in ("waves", "unroll", "xcd_remap", "pipeline", "zigzag", "codes", "temporal"))
    kern = "k_sweep_f64<"
    fetch, nd, kname = _counter_per_dispatch(fetch_dir, kern)
    write, _, _ = _counter_per_dispatch(write_dir, kern)
    cfetch, _, _ = _counter_per_dispatch(copy_fetch_dir, "copyBuffer", largest=True)
    cwrite, _, _ = _counter_per_dispatch(copy_write_dir, "copyBuffer", largest=True)
    nbytes = 1 << 30
    fs, ws = nbytes / (cfetch * 1024), nbytes / (cwrite * 1024)
    entry = {"kernel": kname.replace("(anonymous namespace)::", "").replace("void ", "").replace("rbf::", "").split("(")[0],
             "kernel_source": sweep_source_hash(), "shape": shape,
             "fetch_kib_per_dispatch": round(fetch, 1), "write_kib_per_dispatch": round(write, 1),
             "dispatches": nd, "fetch_scale": round(fs, 5), "write_scale": round(ws, 5),
             "bytes_per_launch": int(fetch * 1024 * fs + write * 1024 * ws),
             "fetch_bytes": int(fetch * 1024 * fs), "write_bytes": int(write * 1024 * ws),
             # algorithmic bytes: 12n + 16 read and 8 written per interior row
             "alg_read_bytes": rf["alg_bytes_per_launch"] - 8 * line["config"]["interior_nodes"],
             "alg_write_bytes": 8 * line["config"]["interior_nodes"],
             "format_bytes": rf["format_bytes_per_launch"]}
    entry["bytes_per_launch"] = entry["fetch_bytes"] + entry["write_bytes"]
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        d = {}
    key = "sweep_f64|cube1M|m4"
    d[key] = entry
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps({key: entry}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--orders", default="4,2,6", help="augmentation orders; the first is the headline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tte", action="store_true", help="skip the time-to-error comparison")
    ap.add_argument("--no-c2", action="store_true", help="skip the 8M-node FP32+refine vs FP64 block")
    ap.add_argument("--no-c4", action="store_true", help="skip the 2M-node adjoint block")
    ap.add_argument("--tte-target", type=float, default=1e-6)
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--record-traffic", nargs=5, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                           "COPY_WRITE_DIR", "BENCH_JSON"),
                    help="write profiles/traffic.json from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (no GPU)")
    ap.add_argument("--workload", default="cube1M",
                    choices=["cube1M", "cube1M_fp32", "cube8M", "cube4M_bands", "cube2M_adjoint", "support_sweep",
                             "order_scan", "mixed_bc", "square10k"],
                    help="cube1M: the benchmark line; the others print their own measurement line")
    ap.add_argument("--mode", default="fp64", choices=["fp64", "fp32_refine"], help="cube8M: iteration mode")
    ap.add_argument("--directions", type=int, default=32, help="cube2M_adjoint: central-difference directions")
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(*args.record_traffic)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    # shapes tuned on MI355X ship with the package; other shapes are tuned on first use
    tuned = os.path.join(ROOT, "paper_2502_12878_amd", "tuned_gfx950.json")
    os.environ.setdefault("RBF_AUTOTUNE_CACHE", tuned if os.path.exists(tuned) else
                          os.path.join(ROOT, "_build", "autotune.json"))
    os.makedirs(os.path.join(ROOT, "_build"), exist_ok=True)
    import torch
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload != "cube1M":
        if args.workload == "cube8M":
            out = run_cube8m(args.mode, args.tte_target)
        elif args.workload == "cube4M_bands":
            out = run_cube4m_bands()
        elif args.workload == "support_sweep":
            out = run_support_sweep()
        elif args.workload == "order_scan":
            out = run_order_scan()
        elif args.workload == "mixed_bc":
            out = run_mixed_bc()
        elif args.workload == "cube1M_fp32":
            out = run_cube1m_fp32()
        elif args.workload == "square10k":
            out = run_square10k()
        else:
            out = run_cube2m_adjoint(directions=args.directions)
        out["device"] = torch.cuda.get_device_name(0)
        print(json.dumps(out))
        return
    orders = [int(x) for x in args.orders.split(",") if x]
    per_order = {}
    head = None
    for i, m in enumerate(orders):
        _progress(f"cube1M m={m}: setup and {args.steps} timed steps")
        s = setup_problem(m, keep_fp32=(i == 0 and not args.no_tte))
        wl = s["wl"]
        nint = int((s["typ"] == 0).sum())
        wall, per_sweep, nsw, rep, warm_run = time_sweeps(s, args.steps, args.warmup)
        bytes_per_update = 12 * wl.n + 24
        alg_bytes = bytes_per_update * nint
        info = s["p"].operator_info()
        entry = {"m": m, "n": wl.n, "interior_nodes": nint, "node_updates_per_s": nint * args.steps / wall,
                 "ms_per_step": 1e3 * wall / args.steps, "kernel_ms_per_sweep": 1e3 * per_sweep,
                 "warmup_steps_run": warm_run,
                 "alg_bytes_per_update": bytes_per_update, "alg_GBps": alg_bytes / per_sweep / 1e9,
                 "hbm_frac": alg_bytes / per_sweep / 1e9 / PEAK_HBM_GBS, "res_final": rep["res_final"],
                 "format_bytes_per_sweep": info["stream_bytes_f64"],
                 "format_GBps": info["stream_bytes_f64"] / per_sweep / 1e9,
                 "sweep_shape": {k[4:]: v for k, v in info.items() if k.startswith("f64_")},
                 "coded_slices_frac": round(info["coded_slices"] / max(1, info["slices"]), 4),
                 "setup": {k: round(v, 3) for k, v in s["setup"].items()}}
        if i == 0:
            entry["event_windows"] = sweep_windows(s)
        per_order[m] = entry
        if i == 0:
            head = (s, entry, wall, per_sweep, nsw)
        else:
            s["p"].close()
    s, entry, wall, per_sweep, nsw = head
    wl = s["wl"]
    key = f"sweep_f64|cube1M|m{wl.m}"
    sh = entry["sweep_shape"]
    traffic = stored_traffic(key, ",".join(str(sh[k]) for k in ("waves", "unroll", "xcd_remap", "pipeline",
                                                                "zigzag", "codes", "temporal")))
    alg_bytes = entry["alg_bytes_per_update"] * entry["interior_nodes"]
    roofline = {"bound": "hbm", "achieved": round(alg_bytes / per_sweep / 1e9, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(alg_bytes / per_sweep / 1e9 / PEAK_HBM_GBS, 4),
                "traffic": traffic,
                "traffic_GBps": round(traffic / per_sweep / 1e9, 1) if traffic else None,
                "kernel": "k_sweep_f64", "alg_bytes_per_launch": alg_bytes,
                "avg_launch_ms": round(1e3 * per_sweep, 5), "launches_timed": nsw,
                "format_bytes_per_launch": entry["format_bytes_per_sweep"],
                "format_frac": round(entry["format_GBps"] / PEAK_HBM_GBS, 4), "sweep_shape": entry["sweep_shape"]}
    tte = None
    if not args.no_tte:
        _progress("cube1M: time to L-inf error, FP64 and FP32 + refinement")
        tte = time_to_error(s, args.tte_target)
        info = s["p"].operator_info()
        tte["fp32_sweep_shape"] = {k[4:]: v for k, v in info.items() if k.startswith("f32_")}
        tte["fp32_format_bytes_per_sweep"] = info["stream_bytes_f32"]
        r = tte["fp32_refine"]
        if r["steps"]:
            # device time per inner step of the refinement run (its outer
            # FP64 residuals included, one per 500 steps) against 8n + 12 bytes
            per32 = r["device_s"] / r["steps"]
            alg32 = (8 * wl.n + 12) * entry["interior_nodes"]
            tte["fp32_ms_per_inner_step"] = round(1e3 * per32, 5)
            tte["fp32_alg_GBps"] = round(alg32 / per32 / 1e9, 1)
            tte["fp32_hbm_frac"] = round(alg32 / per32 / 1e9 / PEAK_HBM_GBS, 4)
    cpu = None
    if not args.no_cpu:
        _progress("CPU baseline: the oracle's OpenMP sweep on the cube1M operator")
        cpu = cpu_baseline(s)
    s["p"].close()
    del s
    torch.cuda.empty_cache()
    c2 = None
    if not args.no_c2:
        _progress("cube8M: FP64 and FP32 + refinement steps")
        c2 = run_c2_block()
    c4 = None
    if not args.no_c4:
        _progress("cube2M adjoint: gradient vs central differences and the oracle")
        c4 = run_cube2m_adjoint()
    out = {"metric": "sweep node-updates/s + HBM GB/s; time to L-inf err 1e-6, FP32+refine vs FP64",
           "value": entry["node_updates_per_s"], "unit": "node-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": entry["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "scaling_note": "one GPU only (no multi-GPU path); a shard would hold one "
                                              "fixed-size block of rows per GPU",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"cube1M: 3D 100^3 jittered grid (seed 1), m={wl.m}, n={wl.n}, "
                                  f"dt={wl.alpha}*h^2/6, FP64 explicit sweep",
                      "interior_nodes": entry["interior_nodes"], "parallelism": "single GPU"},
           "roofline": roofline, "cpu_baseline": cpu,
           "orders": {str(k): v for k, v in per_order.items()}, "time_to_error": tte,
           "cube8M_fp32_refine_vs_fp64": c2, "cube2M_adjoint": c4,
           "stream_ceiling": stream_ceiling(), "ell_layout": int(os.environ.get("RBF_ELL_LAYOUT", "1")),
           "device": torch.cuda.get_device_name(0)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
