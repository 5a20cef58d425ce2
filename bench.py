"""Benchmark: PDIP time-step ms and Newton-step solve ms at 2^20 unknowns.

One step is one frictional-contact time step of the whole hot path on the
GPU: contact detection and ordering, assembly of N and r, the PDIP loop
(per Newton iteration: barrier blocks, block-Jacobi + QTT compression and
Newton-Schulz inverse update, FGMRES to 1e-8), and integration.  Workload:
the seeded rectangular hopper fill of 131,072 spheres (radius uniform in
[0.8, 1.2] cm, mu = 0.4, h = 1e-3 s), ~3.4e5 contacts padded to 2^20.

    python bench.py [--steps K] [--warmup W] [--precision f64|f32|bf16]

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def spmv_bytes(nnzb, n):
    """Algorithmic bytes of one BSR3 product: values, block columns, row
    pointers, x gathered once, y written once."""
    nslots = n // 3
    return 72 * nnzb + 4 * nnzb + 4 * (nslots + 1) + 16 * n


def cpu_baseline(precision_note):
    """The oracle's time step on a bounded hopper sample, scaled to 2^20."""
    import numpy as np

    import scenes
    from oracle import pdip

    nx, ny, nz = 8, 4, 32
    sc = scenes.hopper(seed=3, nx=nx, ny=ny, nz=nz)
    t0 = time.perf_counter()
    c, res, gamma, _ = pdip.time_step(sc)
    dt = time.perf_counter() - t0
    full_spheres = 64 * 64 * 32
    scale = full_spheres / sc.M
    cores = os.cpu_count() or 1
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] + [1])
    except Exception:
        pass
    return {
        "value": dt * 1e3 * scale,
        "unit": "ms",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"one PDIP time step of a {nx}x{ny}x{nz} hopper fill "
                   f"({sc.M} spheres, {c.nc} contacts, {res.iterations} PDIP "
                   f"iterations, SuperLU Newton solves) in {dt:.1f} s, scaled "
                   f"linearly by {scale:.0f} to 131,072 spheres"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="f32", choices=["f64", "f32", "bf16"])
    ap.add_argument("--rmax", type=int, default=32)
    ap.add_argument("--rmax-s", type=int, default=16)
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--ns-iters", type=int, default=6)
    ap.add_argument("--ns-iters-hot", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scene", default="hopper")
    ap.add_argument("--qtt-mode", type=int, default=2, choices=[0, 1, 2],
                    help="0 block-Jacobi only, 1 QTT inverse always, 2 per-step trial")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the "
              "multi-GPU layout is a design, not a run", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("RANK", "0")) != 0:
        return

    import numpy as np
    import torch

    import scenes
    from paper_1808_02558_amd import binding

    torch.cuda.set_device(0)
    sc = scenes.make_scene(a.scene)
    ctx = binding.Context(precision=a.precision, qtt_rmax=a.rmax,
                          qtt_rmax_s=a.rmax_s, qtt_eps=a.eps, solve_mode=1,
                          solve_tol=1e-8, fgmres_restart=a.restart,
                          fgmres_maxit=3000, ns_iters=a.ns_iters,
                          ns_iters_hot=a.ns_iters_hot, qtt_mode=a.qtt_mode)

    def dev(x):
        return torch.from_numpy(np.ascontiguousarray(x)).cuda()

    ctx.qtp_set_bodies(dev(sc.x), dev(sc.v), dev(sc.w), dev(sc.radius), dev(sc.mass))
    ctx.qtp_set_walls(sc.planes)
    ctx.qtp_set_params(sc.mu, sc.h, sc.delta, sc.gravity, sc.log2n)
    n = 1 << sc.log2n

    stats = []
    recs = []
    for i in range(a.warmup):
        rc, st = ctx.qtp_step()
        print(f"warmup step {i}: {st.n_contacts} contacts, {st.pdip_iterations} PDIP "
              f"its, {st.fgmres_iterations} FGMRES its, {st.ms_total:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ctx.qtp_profile(True)
    t0 = time.perf_counter()
    for i in range(a.steps):
        rc, st = ctx.qtp_step()
        stats.append(st)
        recs.extend(ctx.qtp_get_newton_log())
        print(f"step {i}: {st.n_contacts} contacts, {st.pdip_iterations} PDIP its "
              f"(converged {st.converged}), {st.fgmres_iterations} FGMRES its "
              f"(max {st.max_fgmres}), qtt_used {st.qtt_used}, precond {st.ms_precond:.1f} ms, solves "
              f"{st.ms_solve:.1f} ms, total {st.ms_total:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    # dominant Newton-step kernel: the BSR3 sparse product
    sp_ms, sp_n = ctx.qtp_get_kernel_time("bsr_spmv")
    qa_ms, qa_n = ctx.qtp_get_kernel_time("qtt_apply")
    cg_ms, cg_n = ctx.qtp_get_kernel_time("cgs2")
    ctx.qtp_profile(False)
    try:
        ranks_x = ctx.qtp_get_qtt_ranks(1)
        ranks_s = ctx.qtp_get_qtt_ranks(0)
    except binding.QtpError:  # block-Jacobi only: no QTT was built
        ranks_x = ranks_s = None
    pst = ctx.qtp_get_precond_stats()
    _, _, valN, _ = ctx.qtp_get_qp(sc.log2n)
    nnzb = valN.numel() // 9
    ctx.close()

    solve_ms = float(np.median([r.solve_ms for r in recs]))
    its = np.array([r.fgmres_iterations for r in recs])
    sms = np.array([r.solve_ms for r in recs])
    print("newton solves: iterations " + " ".join(str(int(i)) for i in its),
          file=sys.stderr, flush=True)
    fg = [s.fgmres_iterations / max(s.pdip_iterations, 1) for s in stats]
    sp_avg = sp_ms / max(sp_n, 1)
    sp_bytes = spmv_bytes(nnzb, n)
    achieved = sp_bytes / (sp_avg * 1e-3) / 1e9 if sp_n else None
    out = {
        "metric": "Newton-step solve ms & PDIP time-step ms at 2^20 unknowns, "
                  "1e-8 residual",
        "value": ms_per_step,
        "unit": "ms",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{a.scene}: {sc.M} spheres, 2^{sc.log2n} unknowns, "
                        f"mu {sc.mu}, h {sc.h}",
            "qtt_cores": a.precision, "qtt_eps": a.eps, "qtt_rmax": a.rmax,
            "qtt_rmax_s": a.rmax_s, "fgmres": f"FGMRES({a.restart}) to 1e-8",
            "pdip_gap_tol": 1e-8, "qtt_mode": a.qtt_mode,
        },
        "qtt_used": [s.qtt_used for s in stats],
        "trial_iterations": {"qtt": [s.qtt_trial_iterations for s in stats],
                             "block_jacobi": [s.plain_trial_iterations for s in stats]},
        "newton_solve_ms": solve_ms,
        "qtt_ranks_last": {"X": ranks_x, "S": ranks_s,
                           "ns_iterations": pst.ns_iterations,
                           "probe_residual": pst.probe_residual},
        "newton_solves": {
            "count": int(len(recs)),
            "ms": {"median": solve_ms, "p90": float(np.percentile(sms, 90)),
                   "max": float(sms.max()), "mean": float(sms.mean())},
            "fgmres_iterations": {"median": float(np.median(its)),
                                  "p90": float(np.percentile(its, 90)),
                                  "max": int(its.max()), "mean": float(its.mean())},
            "max_rel_residual": float(max(r.rel_residual for r in recs)),
        },
        "pdip_iterations": [s.pdip_iterations for s in stats],
        "fgmres_iterations_per_newton": fg,
        "contacts": [s.n_contacts for s in stats],
        "ms_split": {
            "detect": float(np.mean([s.ms_detect for s in stats])),
            "assemble": float(np.mean([s.ms_assemble for s in stats])),
            "precond": float(np.mean([s.ms_precond for s in stats])),
            "solve": float(np.mean([s.ms_solve for s in stats])),
            "pdip_total": float(np.mean([s.ms_pdip for s in stats])),
            "integrate": float(np.mean([s.ms_integrate for s in stats])),
        },
        "kernels": {
            "bsr_spmv": {"ms_avg": sp_avg, "launches": sp_n, "bytes": sp_bytes},
            "qtt_apply": {"ms_avg": qa_ms / max(qa_n, 1), "launches": qa_n},
            "cgs2": {"ms_avg": cg_ms / max(cg_n, 1), "launches": cg_n},
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": None, "kernel": "bsr_spmv",
        },
        "cpu_baseline": None,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.precision)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
