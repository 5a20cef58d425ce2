"""Benchmark: PDIP time-step ms and Newton-step solve ms at 2^20 unknowns.

One step is one frictional-contact time step of the whole hot path on the
GPU: contact detection and ordering, assembly of N and r, the PDIP loop
(per Newton iteration: barrier blocks, block-Jacobi factors, the QTT inverse
where the preconditioner mode uses it, FGMRES to 1e-8), and integration.
By default the steps re-use information across time steps as Sec. 3.3 does:
persistent contacts keep their slots and start the PDIP from their previous
normal impulse; the untimed warm-up step starts cold.
Workload: the seeded rectangular hopper fill of 131,072 spheres (radius
uniform in [0.8, 1.2] cm, mu = 0.4, h = 1e-3 s), ~3.4e5 contacts padded to
2^20 unknowns.

After the timed steps, each form of the method solves the first time step
from the same initial state: the QTT-preconditioned solve with FP64, FP32 and
BF16 cores and the block-Jacobi-only solve; then the learned warm start is
trained on two solved steps and compared with the cold start on the next
step.  Impulses are compared with the FP64 QTT form.

    python bench.py [--steps K] [--warmup W] [--no-forms] [--no-cpu-baseline]

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
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}

# Hardware byte counters of the current bsr3_spmv_kernel on the hopper step
# (two rocprofv3 --pmc passes, FETCH_SIZE then WRITE_SIZE, KiB per dispatch
# averaged over the step), each scaled by what the same counter reads for a
# 256 MiB device-to-device copy in the same program; the command lines are in
# profiles/bsr3_spmv_hopper_2p20_traffic.md.  Reset to None whenever the
# kernel changes until the passes are taken again.
SPMV_COUNTERS = {
    "hopper": {"fetch_kib": 132380.51, "write_kib": 8198.24,
               "copy_fetch_kib": 131088.5, "copy_write_kib": 262144.0,
               "copy_kib": 262144.0},
}


def spmv_traffic(scene):
    c = SPMV_COUNTERS.get(scene)
    if c is None:
        return None
    return 1024.0 * (c["fetch_kib"] * c["copy_kib"] / c["copy_fetch_kib"] +
                     c["write_kib"] * c["copy_kib"] / c["copy_write_kib"])


def spmv_bytes(nnzb, n):
    """Algorithmic bytes of one BSR3 product: values, block columns, row
    pointers, x gathered once, y written once."""
    nslots = n // 3
    return 72 * nnzb + 4 * nnzb + 4 * (nslots + 1) + 16 * n


def qtt_apply_work(ranks, n, prec):
    """Flops (4 N sum_k r_{k-1} r_k) and minimum bytes (x in and y out in
    FP64, the cores once) of one QTT matrix-vector product."""
    pairs = sum(ranks[k] * ranks[k + 1] for k in range(len(ranks) - 1))
    core_bytes = 4 * pairs * {"f64": 8, "f32": 4, "bf16": 2}[prec]
    return 4.0 * n * pairs, 16.0 * n + core_bytes


def cpu_baseline():
    """The oracle's time step on a bounded hopper sample, scaled to 2^20."""
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_context(binding, torch, sc, **cfg):
    import numpy as np

    def dev(x):
        return torch.from_numpy(np.ascontiguousarray(x)).cuda()

    ctx = binding.Context(**cfg)
    ctx.qtp_set_bodies(dev(sc.x), dev(sc.v), dev(sc.w), dev(sc.radius), dev(sc.mass))
    ctx.qtp_set_walls(sc.planes)
    ctx.qtp_set_params(sc.mu, sc.h, sc.delta, sc.gravity, sc.log2n)
    return ctx


def rel_err(g, ref):
    import numpy as np
    return float(np.linalg.norm(g - ref) / np.linalg.norm(ref))


def step_summary(st):
    return {"ms": st.ms_total, "pdip_iterations": st.pdip_iterations,
            "fgmres_iterations": st.fgmres_iterations, "max_fgmres": st.max_fgmres,
            "precond_ms": st.ms_precond, "solve_ms": st.ms_solve,
            "converged": bool(st.converged)}


def qtt_form(binding, torch, sc, base, prec):
    """First time step with the QTT inverse applied at every Newton step."""
    import numpy as np
    ctx = make_context(binding, torch, sc, **dict(base, qtt_mode=1, precision=prec))
    try:
        ctx.qtp_profile(True)
        rc, st = ctx.qtp_step()
        g = ctx.qtp_get_impulses(st.n_contacts).cpu().numpy()
        qa_ms, qa_n = ctx.qtp_get_kernel_time("qtt_apply")
        ranks = ctx.qtp_get_qtt_ranks(1)
        recs = ctx.qtp_get_newton_log()
        ctx.qtp_profile(False)
    finally:
        ctx.close()
    n = 1 << sc.log2n
    out = step_summary(st)
    out["newton_solve_ms_median"] = float(np.median([r.solve_ms for r in recs]))
    if qa_n:
        avg = qa_ms / qa_n
        flops, nbytes = qtt_apply_work(ranks, n, prec)
        tf = flops / (avg * 1e-3) / 1e12
        out["qtt_apply"] = {
            "ms_avg": avg, "launches": qa_n, "ranks_last": ranks, "tflops": tf,
            "frac_of_peak_flops": tf / PEAK_TFLOPS[prec],
            "min_bytes_gbs": nbytes / (avg * 1e-3) / 1e9}
    log(f"form qtt {prec}: {st.pdip_iterations} PDIP its, {st.fgmres_iterations} "
        f"FGMRES its, {st.ms_total:.1f} ms")
    return out, g


def simple_form(binding, torch, sc, cfg, label):
    ctx = make_context(binding, torch, sc, **cfg)
    try:
        rc, st = ctx.qtp_step()
        g = ctx.qtp_get_impulses(st.n_contacts).cpu().numpy()
    finally:
        ctx.close()
    log(f"form {label}: {st.pdip_iterations} PDIP its, {st.fgmres_iterations} FGMRES "
        f"its, {st.ms_total:.1f} ms")
    return step_summary(st), g


def mlp_form(binding, torch, sc, base, train_steps=2, epochs=12, batch=4096, lr=1e-3):
    """Learned warm start: train the network on the solved impulses of the
    first time steps (the library's forward, backward and Adam kernels), then
    solve the next time step cold and from the prediction, for several
    centring parameters t0 and floors on the predicted normal impulse."""
    import numpy as np

    import scenes
    ctx = make_context(binding, torch, sc, **dict(base, warm_start=0))
    try:
        Xs, Ys = [], []
        for _ in range(train_steps):
            nc = ctx.qtp_detect()
            ctx.qtp_assemble()
            Xs.append(ctx.qtp_mlp_features(nc))
            ctx.qtp_pdip_solve()
            Ys.append(ctx.qtp_mlp_targets(nc))
            ctx.qtp_integrate()
        X = torch.cat(Xs)
        Y = torch.cat(Ys)
        params = np.concatenate([p.reshape(-1) for p in scenes.tensors.mlp_init(
            [11, 128, 128, 128, 3], seed=1000)]).astype(np.float32)
        ctx.qtp_mlp_set_params(torch.from_numpy(params).cuda())
        ctx.qtp_mlp_fit_normalization(X)
        rows = X.shape[0]
        perm = torch.from_numpy(np.random.default_rng(0).permutation(rows)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        first = last = None
        nsteps = 0
        for _ in range(epochs):
            for b0 in range(0, rows, batch):
                idx = perm[b0:b0 + batch]
                loss = ctx.qtp_mlp_train_step(X[idx].contiguous(), Y[idx].contiguous(),
                                              lr=lr)
                first = loss if first is None else first
                last = loss
                nsteps += 1
        torch.cuda.synchronize()
        train_ms = (time.perf_counter() - t0) * 1e3
        # held-out step: cold first (also gives the held-out targets)
        nc = ctx.qtp_detect()
        ctx.qtp_assemble()
        Xh = ctx.qtp_mlp_features(nc)
        rc_c, cold = ctx.qtp_pdip_solve()
        gc = ctx.qtp_get_impulses(nc).cpu().numpy()
        Yh = ctx.qtp_mlp_targets(nc)
        Ph = ctx.qtp_mlp_forward(Xh)
        err = (Ph - Yh).double()
        loaded = Yh[:, 0] > float(np.log(1e-3))
        held = {"mse": float((err ** 2).mean()),
                "rms_log_gn_loaded": float((err[loaded, 0] ** 2).mean().sqrt()),
                "rms_log_gn_unloaded": float((err[~loaded, 0] ** 2).mean().sqrt()),
                "loaded_fraction": float(loaded.double().mean())}
        trials = []
        for t0w in (1.0, 10.0, 100.0):
            for floor in (0.0, 1e-3, 1e-2, 1e-1):
                ctx.qtp_set_config(warm_start=2, warm_t0=t0w, warm_floor=floor)
                rc_w, warm = ctx.qtp_pdip_solve()
                gw = ctx.qtp_get_impulses(nc).cpu().numpy()
                trials.append({"t0": t0w, "floor": floor,
                               "pdip_iterations": (warm.warm_iterations
                                                   if warm.warm_fallback
                                                   else warm.pdip_iterations),
                               "fallback": bool(warm.warm_fallback),
                               "ms": warm.ms_pdip,
                               "impulse_rel_diff_vs_cold": rel_err(gw, gc)})
        ctx.qtp_set_config(warm_start=0)
    finally:
        ctx.close()
    best = min(trials, key=lambda t: t["ms"])
    log(f"form mlp: cold {cold.pdip_iterations} PDIP its {cold.ms_pdip:.1f} ms; best "
        f"warm t0 {best['t0']} floor {best['floor']}: {best['pdip_iterations']} its "
        f"{best['ms']:.1f} ms (fallback {best['fallback']}); loss {first:.4f} -> "
        f"{last:.4f}, held-out mse {held['mse']:.4f}")
    return {
        "training": {"rows": int(rows), "steps_of_data": train_steps, "epochs": epochs,
                     "adam_steps": nsteps, "batch": batch, "lr": lr,
                     "loss_first": first, "loss_last": last, "ms": train_ms},
        "held_out_step": {
            "prediction": held,
            "cold": {"pdip_iterations": cold.pdip_iterations,
                     "fgmres_iterations": cold.fgmres_iterations, "ms": cold.ms_pdip,
                     "converged": bool(cold.converged)},
            "warm_trials": trials,
            "best_warm": best},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="f32", choices=["f64", "f32", "bf16"])
    ap.add_argument("--rmax", type=int, default=32)
    ap.add_argument("--rmax-s", type=int, default=16)
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--ns-iters", type=int, default=6)
    ap.add_argument("--ns-iters-hot", type=int, default=2)
    ap.add_argument("--qtt-mode", type=int, default=2, choices=[0, 1, 2],
                    help="0 block-Jacobi only, 1 QTT inverse always, 2 per-step trial")
    ap.add_argument("--scene", default="hopper")
    ap.add_argument("--slot-mode", type=int, default=1, choices=[0, 1],
                    help="1: contacts keep their slots across time steps")
    ap.add_argument("--warm-start", type=int, default=1, choices=[0, 1, 3],
                    help="1: previous step's normal impulses of persistent contacts; "
                         "3: their whole previous impulses")
    ap.add_argument("--warm-t0", type=float, default=1.0)
    ap.add_argument("--warm-floor", type=float, default=0.0)
    ap.add_argument("--warm-maxit", type=int, default=40)
    ap.add_argument("--pdip-maxit", type=int, default=100)
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (the "
                         "reference kernel for scaling hardware byte counters)")
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
    if a.copy_probe_mb:
        src = torch.ones(a.copy_probe_mb << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {a.copy_probe_mb} MiB device to device")
        del src, dst
    sc = scenes.make_scene(a.scene)
    base = dict(qtt_rmax=a.rmax, qtt_rmax_s=a.rmax_s, qtt_eps=a.eps, solve_mode=1,
                solve_tol=1e-8, fgmres_restart=a.restart, fgmres_maxit=3000,
                ns_iters=a.ns_iters, ns_iters_hot=a.ns_iters_hot,
                pdip_maxit=a.pdip_maxit)
    ctx = make_context(binding, torch, sc,
                       **dict(base, precision=a.precision, qtt_mode=a.qtt_mode,
                              slot_mode=a.slot_mode, warm_start=a.warm_start,
                              warm_t0=a.warm_t0, warm_floor=a.warm_floor,
                              warm_maxit=a.warm_maxit))
    n = 1 << sc.log2n

    stats, recs = [], []
    g_first = None
    for i in range(a.warmup):
        rc, st = ctx.qtp_step()
        if i == 0:
            g_first = ctx.qtp_get_impulses(st.n_contacts).cpu().numpy()
        log(f"warmup step {i}: {st.n_contacts} contacts, {st.pdip_iterations} PDIP "
            f"its, {st.fgmres_iterations} FGMRES its, {st.ms_total:.1f} ms")
    torch.cuda.synchronize()
    ctx.qtp_profile(True)
    t0 = time.perf_counter()
    for i in range(a.steps):
        rc, st = ctx.qtp_step()
        stats.append(st)
        recs.extend(ctx.qtp_get_newton_log())
        log(f"step {i}: {st.n_contacts} contacts, {st.pdip_iterations} PDIP its "
            f"(converged {st.converged}, start {st.warm_started}, fallback "
            f"{st.warm_fallback}, kept slots {st.persistent_contacts}), "
            f"{st.fgmres_iterations} FGMRES its "
            f"(max {st.max_fgmres}), qtt_used {st.qtt_used}, precond "
            f"{st.ms_precond:.1f} ms, solves {st.ms_solve:.1f} ms, total "
            f"{st.ms_total:.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    kernels = {}
    for name in ("bsr_spmv", "arnoldi_next", "arnoldi_dots", "arnoldi_orth",
                 "qtt_apply"):
        ms, cnt = ctx.qtp_get_kernel_time(name)
        kernels[name] = {"ms_avg": ms / max(cnt, 1), "launches": cnt}
    ctx.qtp_profile(False)
    try:
        ranks_x = ctx.qtp_get_qtt_ranks(1)
        ranks_s = ctx.qtp_get_qtt_ranks(0)
    except binding.QtpError:  # block-Jacobi only: no QTT was built
        ranks_x = ranks_s = None
    _, _, valN, _ = ctx.qtp_get_qp(sc.log2n)
    nnzb = valN.numel() // 9
    ctx.close()

    its = np.array([r.fgmres_iterations for r in recs])
    sms = np.array([r.solve_ms for r in recs])
    log("newton solves: iterations " + " ".join(str(int(i)) for i in its))
    # dominant Newton-step kernel: the BSR3 sparse product
    sp = kernels["bsr_spmv"]
    sp["bytes"] = spmv_bytes(nnzb, n)
    achieved = sp["bytes"] / (sp["ms_avg"] * 1e-3) / 1e9 if sp["launches"] else None
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
            "qtt_mode": a.qtt_mode, "qtt_cores": a.precision, "qtt_eps": a.eps,
            "qtt_rmax": a.rmax, "qtt_rmax_s": a.rmax_s, "slot_mode": a.slot_mode,
            "warm_start": a.warm_start, "warm_t0": a.warm_t0,
            "warm_floor": a.warm_floor, "warm_maxit": a.warm_maxit,
            "fgmres": f"FGMRES({a.restart}) to 1e-8", "pdip_gap_tol": 1e-8,
        },
        "newton_solve_ms": float(np.median(sms)),
        "newton_solves": {
            "count": int(len(recs)),
            "ms": {"median": float(np.median(sms)), "p90": float(np.percentile(sms, 90)),
                   "max": float(sms.max()), "mean": float(sms.mean())},
            "fgmres_iterations": {"median": float(np.median(its)),
                                  "p90": float(np.percentile(its, 90)),
                                  "max": int(its.max()), "mean": float(its.mean())},
            "max_rel_residual": float(max(r.rel_residual for r in recs)),
        },
        "qtt_used": [s.qtt_used for s in stats],
        "trial_iterations": {"qtt": [s.qtt_trial_iterations for s in stats],
                             "block_jacobi": [s.plain_trial_iterations for s in stats]},
        "qtt_ranks_last": {"X": ranks_x, "S": ranks_s},
        "pdip_iterations": [s.pdip_iterations for s in stats],
        "contacts": [s.n_contacts for s in stats],
        "ms_split": {
            "detect": float(np.mean([s.ms_detect for s in stats])),
            "assemble": float(np.mean([s.ms_assemble for s in stats])),
            "precond": float(np.mean([s.ms_precond for s in stats])),
            "solve": float(np.mean([s.ms_solve for s in stats])),
            "pdip_total": float(np.mean([s.ms_pdip for s in stats])),
            "integrate": float(np.mean([s.ms_integrate for s in stats])),
        },
        "kernels": kernels,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": spmv_traffic(a.scene), "kernel": "bsr_spmv",
        },
        "forms": None,
        "cpu_baseline": None,
    }
    if not a.no_forms:
        forms = {}
        f64, g64 = qtt_form(binding, torch, sc, base, "f64")
        forms["qtt_f64"] = f64
        for prec in ("f32", "bf16"):
            f, g = qtt_form(binding, torch, sc, base, prec)
            f["impulse_rel_err_vs_qtt_f64"] = rel_err(g, g64)
            forms[f"qtt_{prec}"] = f
        f, g = simple_form(binding, torch, sc, dict(base, qtt_mode=0), "block_jacobi")
        f["impulse_rel_err_vs_qtt_f64"] = rel_err(g, g64)
        forms["block_jacobi"] = f
        if g_first is not None:
            forms["headline_first_step_impulse_rel_err_vs_qtt_f64"] = rel_err(g_first, g64)
        forms["mlp_warm_start"] = mlp_form(binding, torch, sc, dict(base, qtt_mode=0))
        out["forms"] = forms
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
