"""Tune the sweep shapes (and weight-solver panels) of the benchmark workloads
on the current GPU and store them in an autotuner cache file.

    RBF_AUTOTUNE_CACHE=<file> RBF_AUTOTUNE_FORCE=1 python -m paper_2502_12878_amd.tune_workloads

The package ships the result for MI355X as ``tuned_gfx950.json``; the
benchmark reads it so that its sweeps run in a fixed, profiled shape.
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _operators():
    """(label, builder) for every operator the benchmark sweeps."""
    import rbf_inputs as ri

    def grid(name, m=None, keep_fp32=False):
        def build(p):
            wl = ri.workload(name, m=m)
            xd, td = p.build_nodes(wl.dim, wl.side, wl.jitter, wl.seed)
            p.set_nodes(xd, td)
            p.build_stencils(wl.n)
            p.compute_weights(wl.m, keep_fp32=keep_fp32)
        return build

    def bands(p):
        wl = ri.workload("cube4M_bands")
        xyz, typ = wl.nodes()
        m, n = ri.order_bands(3, xyz, typ, wl.h)
        xd, td = p.build_nodes(3, wl.side, wl.jitter, wl.seed)
        p.set_nodes(xd, td)
        p.build_stencils(n_per_node=n)
        p.compute_weights(m_per_node=m)

    def mixed(p):
        xyz, typ, normals = ri.mixed_bc_grid(3, 100, 0.3, 5)
        p.set_nodes(xyz, typ)
        p.set_normals(normals)
        p.build_stencils(70)
        p.compute_weights(4)

    def cube(side, m, n):
        def build(p):
            xd, td = p.build_nodes(3, side, 0.3, 1)
            p.set_nodes(xd, td)
            p.build_stencils(n)
            p.compute_weights(m)
        return build

    def adjoint(p):
        grid("cube2M_adjoint")(p)
        p.autotune()
        # one short adjoint builds the transposed operator and tunes its gather
        import torch
        N = p.sizes["N"]
        p.adjoint_f(torch.zeros(N, dtype=torch.float64, device=p.device), 2, 1, 1e-6)

    ops = [("cube1M m=4 (FP64 + FP32)", grid("cube1M", 4, True)), ("cube1M m=2", grid("cube1M", 2)),
           ("cube1M m=6", grid("cube1M", 6)), ("cube8M (FP64 + FP32)", grid("cube8M", keep_fp32=True)),
           ("cube4M bands", bands), ("cube2M adjoint + transposed gather", adjoint),
           ("mixed boundary 100^3", mixed)]
    ops += [(f"cube1M m=2 n={n}", cube(100, 2, n)) for n in (30, 40, 60, 80, 100, 130, 168)]
    ops += [(f"cube side {s} m={m}", cube(s, m, 2 * ri.num_monomials(3, m))) for s in (68,) for m in (2, 4, 6)]
    return ops


def main():
    if not os.environ.get("RBF_AUTOTUNE_CACHE"):
        sys.exit("set RBF_AUTOTUNE_CACHE to the cache file to write")
    from paper_2502_12878_amd import Problem
    for label, build in _operators():
        t0 = time.perf_counter()
        p = Problem(0)
        build(p)
        p.autotune()
        info = p.operator_info()
        shape = [info[f"f64_{k}"] for k in ("waves", "unroll", "xcd_remap", "pipeline", "zigzag", "codes")]
        print(f"{label}: FP64 sweep shape {shape} ({time.perf_counter() - t0:.1f} s)", flush=True)
        p.close()


if __name__ == "__main__":
    main()
