"""Benchmark: fast directional Burton-Miller mat-vecs per second on one GPU.

One "step" is one full sound-hard Burton-Miller H mat-vec through the C ABI
(near-field P2P, S2M, M2M, M2L, L2L, L2T and, when the plan has elements,
the near-field correction), on seeded random complex densities already
resident in HBM.  Plan construction is not timed.

Beside the headline rate the run reports the FP32 far/near-field mat-vec rate
and its difference from FP64, and the GMRES time to a relative residual of
1e-4 for a plane wave: plain FP64 against FP32 with the block-Jacobi plus
learned coupling preconditioner (network trained here on small surfaces at the
same points per wavelength; training and preconditioner set-up are reported
separately).

Prints one JSON line (rank 0) with the metric, the roofline of the dominant
kernel and the oracle's CPU baseline on a bounded sample of rows.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# batched workload: uneven instances (sphere / ellipsoid / star), N ~ U[10k, 100k],
# kD ~ U[5, 60], FP32 far and near field, all instances in one graph launch
BATCH = {"c3": (64, 2, (10_000, 100_000), (5.0, 60.0))}

# learned-preconditioner evaluation: star/ellipsoid training surfaces at
# kD ~ U[20, 80], held-out surfaces at kD = 50, FP32 GMRES to 1e-4
LEARNED = {"c4": {"train": 96, "held_out": 50, "n_split": 32, "kd_train": (20.0, 80.0), "kd_test": 50.0,
                  "seed_train": 3, "seed_test": 4, "krylov_steps": 20}}

# radiation of a pulsating unit sphere (q = du/dn = 1, exact u = 1/(1 - ik)):
# k = 2 pi ... 32 pi with elements of size about lambda / 5 (8 n^2 octahedral
# elements, n = round(sqrt(720 (k / 2 pi)^2 / 8)): 648 ... 184,832 elements)
RADIATION = {"radiation": [2 * math.pi * f for f in (1, 2, 4, 8, 16)]}

# the summation of Table 1 (section 5.1): (octahedral n, k / pi, eps) about
# 20 nodes per wavelength, N = 73,008 ... 4,732,608 (the paper's 73,728 ...
# 4,718,592), improved method and the original one it is compared with
TABLE1 = {"table1": [(39, 8, 1e-4), (39, 8, 1e-6), (39, 8, 1e-8), (78, 16, 1e-4), (78, 16, 1e-6),
                     (157, 32, 1e-4), (157, 32, 1e-6), (314, 64, 1e-4)]}

WORKLOADS = {
    # name: (octahedral split n, k, eps, description)
    "c1": (8, 5.0, 1e-4, "unit sphere, 512 quadratic triangles, N=3072, k=5 (kD=10), eps=1e-4"),
    "c2": (64, 50.0, 1e-4, "unit sphere, 32768 quadratic triangles, N=196608, k=50 (kD=100), eps=1e-4, leaf<=64"),
    "c5": (289, 500.0, 1e-4, "unit sphere, 668168 quadratic triangles, N=4009008, k=500 (kD=1000), eps=1e-4"),
    # elongated body standing in for the paper's large non-spherical model: a
    # 1:1:8 prolate ellipsoid (D = 16) at kD = 1000; raw H sum (no elements)
    "f4": (192, 62.5, 1e-4, "prolate ellipsoid 1:1:8 (D=16), 294912 quadratic triangles, N=1769472, "
                            "k=62.5 (kD=1000), eps=1e-4, raw H sum"),
}
ELONGATED = {"f4": 8.0}

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (vector and matrix)
PEAK_HBM_GBS = 8000.0
# FP64 operations of one H-kernel pair in the P2P kernel, counted from its
# source with a fused multiply-add as two: position differences 3, r^2 5,
# r and kr 2, sin and cos of kr 40 (reduction 7, two Horner polynomials 33),
# G 3, the two normal projections and n_x.n_y 17, the kernel combination 26,
# density product and accumulation 8, plus one reciprocal square root
P2P_FLOPS_PER_PAIR = 110
# one kernel evaluation at a check point in S2M (E_up = dG/dn_y) or L2T
# (E_dn = G + alpha dG/dn_x), counted the same way: r and 1/r 8, sin and cos
# 40, G and the normal factor about 20, accumulation 8
EVAL_FLOPS = 76


def m2l_work(plan_stats: dict) -> tuple[float, float]:
    """Algorithmic FP64 flops and HBM bytes of the M2L phase of one mat-vec:
    a dense compressed operator costs 8 s^2 real flops per pair, a rank-r
    factorised one 16 r s; the minimum bytes count each unique operator, each
    source slot and each target slot once."""
    flops = sum(L["m2l_flops"] for L in plan_stats["levels"])
    byts = sum(L["m2l_min_bytes"] for L in plan_stats["levels"])
    return flops, byts


def phase_rooflines(st: dict, phases: dict) -> dict:
    """Achieved rates of the other far-field phases against the peak that
    bounds them: M2M and L2L apply small dense operators to slots (matrix
    cores when their flops per minimum byte -- unique operators, input and
    output slots once -- exceed the machine balance, else HBM); S2M and L2T
    evaluate kernels between leaf points and check points and apply W (FP64
    vector ALU)."""
    out = {}
    for name in ("m2m", "l2l"):
        byts = sum(L[f"{name}_min_bytes"] for L in st["levels"])
        flops = sum(L[f"{name}_flops"] for L in st["levels"])
        ms = phases[name]
        gbs = byts / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        tf = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        # bound by arithmetic intensity against the machine balance (flop per byte)
        if byts > 0 and flops / byts > PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9):
            out[name] = {"bound": "mfma", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / PEAK_FP64_TFLOPS, "algorithmic_bytes": byts, "flops": flops, "gbs": gbs}
        else:
            out[name] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": gbs / PEAK_HBM_GBS, "algorithmic_bytes": byts, "flops": flops, "tflops": tf}
    for name in ("s2m", "l2t"):
        flops = EVAL_FLOPS * st[f"{name}_evals"] + st[f"{name}_w_flops"]
        ms = phases[name]
        tf = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        out[name] = {"bound": "alu", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": tf / PEAK_FP64_TFLOPS, "kernel_evals": st[f"{name}_evals"],
                     "flops_per_eval": EVAL_FLOPS, "w_flops": st[f"{name}_w_flops"]}
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bm_h_matvec_sphere_N4009008_k500.md")
TRAFFIC_SOURCES = ("paper_1311_5202_amd/csrc/apply.hip", "paper_1311_5202_amd/csrc/templates.cpp",
                   "paper_1311_5202_amd/csrc/tree.cpp")


def source_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes of the M2L phase of one mat-vec from the committed counter
    profile (FETCH_SIZE x 2 + WRITE_SIZE x 1, the copy-kernel factors), or None
    when the profile is for another workload or the kernels changed since."""
    if workload != "c5" or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if line.startswith("<!-- traffic "):
                rec = json.loads(line[len("<!-- traffic "):].rsplit("-->", 1)[0])
                if rec.get("source_sha256") == source_digest():
                    return rec["m2l_hbm_bytes_per_matvec"]
    return None


def cpu_baseline(pts, nrm, w, u, k, n_rows: int, gpu_rows=None, coupling: float = 1.0):
    """The oracle's dense FP64 H sum timed on a seeded sample of target rows
    and scaled to a full mat-vec.  gpu_rows: {name: full GPU result of the
    same raw H sum}; their relative L2 error on the sample is reported."""
    import numpy as np

    import oracle

    rows = np.sort(np.random.default_rng(7).choice(len(w), n_rows, replace=False))
    oracle.dense_rows(pts[:64], nrm[:64], w[:64], u[:64], k, "H", rows=np.arange(4))  # load + warm
    t0 = time.perf_counter()
    # the H kernel with alpha = i coupling / k, as the plan
    ref = oracle.dense_rows(pts, nrm, w, u, k, "H", rows=rows, coefs=(0.0, 1.0, 1.0, 1j * coupling / k))
    dt = time.perf_counter() - t0
    full = dt * len(w) / n_rows
    out = {"value": 1.0 / full, "unit": "matvec/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"dense FP64 H sum on {n_rows} of {len(w)} target rows ({dt:.1f} s), scaled to a full mat-vec"}
    for name, g in (gpu_rows or {}).items():
        out[f"gpu_{name}_rel_l2_on_sample"] = oracle.rel_l2(g[rows], ref)
    return out


def train_learned(fdb, synth, density: float, coupling: float, epochs: int, log):
    """Train the coupling network on small star-shaped surfaces whose k gives
    the same number of nodes per square wavelength as the benchmark body, with
    the loss weighted by each surface's own GMRES run."""
    import numpy as np

    net = fdb.Net(11)
    plans = []
    t0 = time.perf_counter()
    for s, n in enumerate((10, 12, 14, 16)):
        el = synth.star_surface(n, seed=100 + s)
        pts, nrm, w = fdb.nystrom_nodes(el)
        k = 2 * np.pi * math.sqrt(len(w) / (density * w.sum()))
        plans.append(fdb.build(pts, nrm, w, k, 1e-4, elements=el, corrections=1, coupling=coupling))
    # loss weights from each surface's own block-Jacobi GMRES run (20 steps, plane wave)
    for i, p in enumerate(plans):
        fdb.Net.weight_blocks(p, p.rhs_plane_wave(synth.random_directions(1, 300 + i)[0]), 20)
    first = [net.loss_grad(p)[0] for p in plans]
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(epochs):
        last = [net.train_step(p, 3e-3) for p in plans]
    t_train = time.perf_counter() - t0
    log(f"[bench] learned: loss {[round(v, 1) for v in first]} -> {[round(v, 1) for v in last]} "
        f"({epochs} epochs, {t_train:.1f} s)")
    for p in plans:
        p.close()
    return net, {"shapes": len(plans), "epochs": epochs, "setup_s": t_setup, "train_s": t_train,
                 "loss_first": sum(first), "loss_last": sum(last)}


def gmres_compare(fdb, synth, plan, tol: float, coupling: float, epochs: int, log, maxit: int = 200):
    """Time-to-tol of plain FP64 GMRES and of FP32 GMRES with the learned
    preconditioner on the same plane-wave right-hand side."""
    import numpy as np
    import torch

    rhs = plan.rhs_plane_wave([0.0, 0.0, 1.0])
    out = {"tol": tol}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x64, i64 = plan.solve(rhs, tol, maxit=maxit, restart=maxit, precond=0, raise_on_fail=False)
    torch.cuda.synchronize()
    out["fp64_plain"] = {"iterations": i64["iterations"], "relres": i64["relres"], "status": i64["status"],
                         "seconds": time.perf_counter() - t0}
    log(f"[bench] FP64 plain GMRES: {out['fp64_plain']}")
    w_sum = float(plan._w.sum())
    density = plan.n * (2 * np.pi / plan.k) ** 2 / w_sum
    net, out["training"] = train_learned(fdb, synth, density, coupling, epochs, log)
    t0 = time.perf_counter()
    net.attach(plan)
    torch.cuda.synchronize()
    out["preconditioner_setup_s"] = time.perf_counter() - t0
    for name, pc in (("fp32_block_jacobi", 1), ("fp32_learned", 2)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = plan.solve(rhs, tol, maxit=maxit, restart=maxit, precond=pc, fp32=True, raise_on_fail=False)
        torch.cuda.synchronize()
        out[name] = {"iterations": info["iterations"], "relres": info["relres"], "status": info["status"],
                     "seconds": time.perf_counter() - t0,
                     "rel_diff_vs_fp64": (torch.linalg.norm(x - x64) / torch.linalg.norm(x64)).item()}
        log(f"[bench] {name} GMRES: {out[name]}")
    net.close()
    out["speedup_fp32_learned_vs_fp64_plain"] = out["fp64_plain"]["seconds"] / out["fp32_learned"]["seconds"]
    return out


def learned_main(args, fdb, synth, torch) -> int:
    """Train the coupling network on seeded training surfaces (N = 49,152,
    kD ~ U[20, 80]) with the loss's block weights taken from each surface's
    own block-Jacobi GMRES run (the Krylov vectors of 20 steps for a plane wave
    from a random direction), and for comparison with uniform weights; then
    compare FP32 GMRES to 1e-4 with block-Jacobi alone and with each learned
    coupling on held-out surfaces at kD = 50 (plane waves from seeded random
    directions)."""
    import numpy as np

    cfg = LEARNED[args.workload]
    n_train = args.instances or cfg["train"]
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731

    def surfaces(count, seed, kd_range):
        rng = np.random.default_rng(seed)
        out = []
        for _ in range(count):
            if rng.uniform() < 0.5:
                el = synth.star_surface(cfg["n_split"], int(rng.integers(0, 2**31 - 1)))
            else:
                el = synth.ellipsoid(cfg["n_split"], float(rng.uniform(1.0, 4.0)))
            p = el.reshape(-1, 3)
            D = float(np.max(p.max(0) - p.min(0)))
            out.append((el, float(rng.uniform(*kd_range)) / D))
        return out

    def build(el, k):
        pts, nrm, w = fdb.nystrom_nodes(el)
        return fdb.build(pts, nrm, w, k, 1e-4, elements=el, corrections=1, precision="both", coupling=args.coupling)

    t0 = time.perf_counter()
    train = []
    dirs_tr = synth.random_directions(n_train, cfg["seed_train"] + 200)
    for i, (el, k) in enumerate(surfaces(n_train, cfg["seed_train"], cfg["kd_train"])):
        train.append(build(el, k))
        if (i + 1) % 16 == 0:
            log(f"[bench] built {i + 1}/{n_train} training surfaces ({time.perf_counter() - t0:.0f} s)")
    t_build = time.perf_counter() - t0
    nets = {}
    t_train = {}
    for name in ("uniform", "gmres_weighted"):
        t0 = time.perf_counter()
        if name == "gmres_weighted":
            for p, d in zip(train, dirs_tr):
                fdb.Net.weight_blocks(p, p.rhs_plane_wave(d), cfg["krylov_steps"])
        net = fdb.Net(17)
        first = sum(net.loss_grad(p)[0] for p in train)
        for ep in range(args.epochs):
            last = sum(net.train_step(p, 3e-3) for p in train)
            if (ep + 1) % 50 == 0:
                log(f"[bench] {name}: epoch {ep + 1}, loss {last:.1f}")
        torch.cuda.synchronize()
        t_train[name] = time.perf_counter() - t0
        log(f"[bench] {name} weights: trained on {len(train)} surfaces, loss {first:.1f} -> {last:.1f} "
            f"in {t_train[name]:.1f} s")
        nets[name] = net
    for p in train:
        p.close()
    dirs = synth.random_directions(cfg["held_out"], cfg["seed_test"] + 100)
    rows = []
    for i, (el, k) in enumerate(surfaces(cfg["held_out"], cfg["seed_test"], (cfg["kd_test"], cfg["kd_test"]))):
        plan = build(el, k)
        rhs = plan.rhs_plane_wave(dirs[i])
        plan.solve(rhs, 1e-4, maxit=300, restart=300, precond=1, fp32=True, raise_on_fail=False)  # set-up
        res = {}
        for name, net in (("block_jacobi", None), ("learned_uniform", nets["uniform"]),
                          ("learned_gmres_weighted", nets["gmres_weighted"])):
            if net is not None:
                net.attach(plan)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, info = plan.solve(rhs, 1e-4, maxit=300, restart=300, precond=1 if net is None else 2, fp32=True,
                                 raise_on_fail=False)
            torch.cuda.synchronize()
            res[name] = (info["iterations"], time.perf_counter() - t1, info["status"])
        log(f"[bench] held-out {i}: N={plan.n} k={k:.1f} " + ", ".join(f"{a} {b[:2]}" for a, b in res.items()))
        rows.append(res)
        plan.close()
    mean = lambda key, j: float(np.mean([r[key][j] for r in rows]))  # noqa: E731
    it_bj, it_u, it_w = mean("block_jacobi", 0), mean("learned_uniform", 0), mean("learned_gmres_weighted", 0)
    t_w = mean("learned_gmres_weighted", 1)
    out = {
        "metric": "held-out GMRES time to 1e-4, FP32 FDA, block-Jacobi + learned coupling (GMRES-run weights)",
        "value": t_w,
        "unit": "s",
        "n_gpus": 1,
        "steps": len(rows),
        "warmup": 1,
        "ms_per_step": 1e3 * t_w,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(train)} training surfaces (star/ellipsoid, N={48 * cfg['n_split'] ** 2}, "
                               f"kD~U{list(cfg['kd_train'])}), {cfg['held_out']} held out at kD={cfg['kd_test']}",
                   "alpha": f"{args.coupling:g}i/k", "parallelism": "single GPU"},
        "iterations_block_jacobi": it_bj,
        "iterations_learned_uniform": it_u,
        "iterations_learned_gmres_weighted": it_w,
        "seconds_block_jacobi": mean("block_jacobi", 1),
        "seconds_learned_uniform": mean("learned_uniform", 1),
        "iteration_reduction_gmres_weighted": 1.0 - it_w / it_bj,
        "iteration_reduction_uniform": 1.0 - it_u / it_bj,
        "converged": all(r[n][2] == 0 for r in rows for n in r),
        "train_s": t_train,
        "build_train_s": t_build,
        "roofline": None,
    }
    for net in nets.values():
        net.close()
    print(json.dumps(out), flush=True)
    return 0


def table1_main(args, fdb, synth, torch) -> int:
    """Table 1 (section 5.1): one summation with the Table-1 kernel
    G + alpha dG/dn_y on random densities, for the improved method and the
    original one (original = 1: equivalent densities with uncompressed R+ and
    K, no low-rank M2L).  Reports per case the M2L time, the upward-pass time
    (S2M + M2M), the plan's device memory and operator bytes, and eps_a on
    200 seeded rows against the oracle's dense sums (the CPU leg)."""
    import numpy as np

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    cases = TABLE1[args.workload]
    if args.cases:
        cases = [cases[int(i)] for i in args.cases.split(",")]
    rows = []
    for n_oct, kp, eps in cases:
        el = synth.octa_sphere(n_oct)
        pts, nrm, w = fdb.nystrom_nodes(el)
        k = kp * math.pi
        u_host = synth.random_densities(len(w), 3)
        u = torch.from_numpy(u_host).cuda()
        for original in (0, 1):
            row = {"N": int(len(w)), "k_over_pi": kp, "eps": eps, "method": "original" if original else "improved"}
            try:
                t0 = time.perf_counter()
                plan = fdb.build(pts, nrm, w, k, eps, original=original, coupling=1.0, verbose=1)
                row["build_s"] = time.perf_counter() - t0
            except fdb.FdaError as e:  # operators beyond the chunk kernel's LDS
                row["error"] = str(e)
                rows.append(row)
                log(f"[bench] table1 {row}")
                continue
            out = torch.empty_like(u)
            for _ in range(2):
                plan.matvec(u, "RAW_T1", out=out)
            plan.set_timing(True)
            for _ in range(max(3, args.steps // 4)):
                plan.matvec(u, "RAW_T1", out=out)
            ph = plan.phase_times()
            plan.set_timing(False)
            st = plan.stats()
            row.update({"t_m2l_ms": ph["m2l"], "t_up_ms": ph["s2m"] + ph["m2m"], "t_total_ms": sum(ph.values()),
                        "device_gb": st["device_bytes"] / 1e9, "operator_gb": st["matpool_bytes"] / 1e9,
                        "s_per_level": [L["s"] for L in st["levels"] if L["s"]]})
            got = out.cpu().numpy()
            plan.close()
            if not args.no_cpu_baseline:
                import oracle

                rr = np.sort(np.random.default_rng(7).choice(len(w), 200, replace=False))
                ref = oracle.dense_rows(pts, nrm, w, u_host, k, "T1", rows=rr)
                row["eps_a"] = oracle.rel_l2(got[rr], ref)
            rows.append(row)
            log(f"[bench] table1 {row}")
    # ratios original / improved per case
    ratios = []
    for a, b in zip(rows[::2], rows[1::2]):
        if "t_m2l_ms" in a and "t_m2l_ms" in b:
            ratios.append({"N": a["N"], "eps": a["eps"], "m2l": b["t_m2l_ms"] / a["t_m2l_ms"],
                           "up": b["t_up_ms"] / a["t_up_ms"], "memory": b["device_gb"] / a["device_gb"]})
    imp = [r for r in rows if r["method"] == "improved" and "t_total_ms" in r]
    last = imp[-1]
    out = {
        "metric": "Table-1 summation (section 5.1): improved FDA time per summation at the largest N run",
        "value": last["t_total_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": len(rows),
        "warmup": 2,
        "ms_per_step": last["t_total_ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "unit sphere, ~20 nodes per wavelength, Table-1 kernel G + (i/k) dG/dn_y, "
                               "random densities, improved vs original FDA", "parallelism": "single GPU"},
        "rows": rows,
        "original_over_improved": ratios,
        "roofline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def radiation_main(args, fdb, synth, torch) -> int:
    """Neumann problem of the pulsating sphere for each k of the series:
    right-hand side (S + alpha M) q - alpha q / 2 by fda_rhs_neumann, GMRES on
    the Burton-Miller operator to tol = eps, error against 1/(1 - ik)."""
    import numpy as np

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    rows = []
    eps = args.eps
    for k in RADIATION[args.workload]:
        n = max(2, int(round(math.sqrt(720.0 * (k / (2 * math.pi)) ** 2 / 8.0))))
        el = synth.octa_sphere(n)
        pts, nrm, w = fdb.nystrom_nodes(el)
        t0 = time.perf_counter()
        plan = fdb.build(pts, nrm, w, k, eps, elements=el, corrections=3, coupling=args.coupling)
        t_build = time.perf_counter() - t0
        q = torch.ones(len(w), dtype=torch.complex128, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rhs = plan.rhs_neumann(q)
        x, info = plan.solve(rhs, eps, maxit=500, restart=500, raise_on_fail=False)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        u = x.cpu().numpy()
        ref = 1.0 / (1.0 - 1j * k)  # the closed form the paper quotes (section 5.2)
        err_l2 = float(np.linalg.norm(u - ref) / (abs(ref) * math.sqrt(len(u))))
        err_max = float(np.max(np.abs(u - ref)) / abs(ref))
        row = {"k_over_pi": round(k / math.pi, 6), "n_elem": int(el.shape[0]), "N": int(len(w)),
               "build_s": t_build, "iterations": info["iterations"], "status": info["status"],
               "solve_s": t_solve, "ms_per_iteration": 1e3 * t_solve / max(1, info["iterations"]),
               "rel_err_l2": err_l2, "rel_err_max": err_max,
               "plan_device_gb": plan.stats().get("device_bytes", 0) / 1e9}
        log(f"[bench] radiation {row}")
        rows.append(row)
        plan.close()
    last = rows[-1]
    out = {
        "metric": "pulsating-sphere radiation solve (GMRES to eps) at the largest k of the series",
        "value": last["solve_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": len(rows),
        "warmup": 0,
        "ms_per_step": last["ms_per_iteration"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "pulsating unit sphere, q = 1, k = 2pi..32pi, elements ~lambda/5 "
                               f"(N = {rows[0]['N']}..{last['N']}), eps = GMRES tol = {eps:g}",
                   "alpha": f"{args.coupling:g}i/k", "parallelism": "single GPU"},
        "series": rows,
        "roofline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def batch_main(args, fdb, synth, torch) -> int:
    """Uneven instances: one graph launch applies every instance's FP32
    mat-vec; compared with the same mat-vecs launched one plan at a time."""
    count, seed, n_range, kd_range = BATCH[args.workload]
    count = args.instances or count
    plans = []
    t0 = time.perf_counter()
    for el, k, kind in synth.instance_batch(count, seed, n_range=n_range, kd_range=kd_range):
        pts, nrm, w = fdb.nystrom_nodes(el)
        plans.append(fdb.build(pts, nrm, w, k, 1e-4, elements=el, corrections=1, precision="both",
                               coupling=args.coupling))
        print(f"[bench] instance {len(plans)}/{count}: {kind} N={len(w)} k={k:.1f}", file=sys.stderr, flush=True)
    t_build = time.perf_counter() - t0
    n_tot = sum(p.n for p in plans)
    us = [torch.from_numpy(synth.random_densities(p.n, i)).cuda() for i, p in enumerate(plans)]
    outs = [torch.empty_like(u) for u in us]
    batch = fdb.Batch(plans)

    def run_batched():
        batch.matvec(us, "BM_H", outs=outs, fp32=True)

    def run_sequential():
        for p, u, o in zip(plans, us, outs):
            p.matvec(u, "BM_H", out=o, fp32=True)

    res = {}
    for name, fn in (("sequential", run_sequential), ("batched", run_batched)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / args.steps
        print(f"[bench] {name}: {1e3 * res[name]:.2f} ms per pass over {count} instances", file=sys.stderr,
              flush=True)
    dt = res["batched"]
    out = {
        "metric": "FDA instance mat-vecs/s (uneven batch, one graph launch)",
        "value": count / dt,
        "unit": "instance-matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{count} instances (sphere/ellipsoid/star), N~U{list(n_range)}, "
                               f"kD~U{list(kd_range)}, eps=1e-4, BM_H, FP32 far and near field",
                   "total_N": n_tot, "alpha": f"{args.coupling:g}i/k", "parallelism": "single GPU"},
        "sequential_ms_per_step": 1e3 * res["sequential"],
        "speedup_vs_sequential_launches": res["sequential"] / dt,
        "build_s": t_build,
        "roofline": None,
    }
    batch.close()
    for p in plans:
        p.close()
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=os.environ.get("FDBEM_WORKLOAD", "c5"),
                    choices=sorted(WORKLOADS) + sorted(BATCH) + sorted(LEARNED) + sorted(RADIATION) + sorted(TABLE1))
    ap.add_argument("--cases", default="", help="table1 workload: comma-separated case indices (default: all)")
    ap.add_argument("--eps", type=float, default=1e-4, help="radiation workload: FDA eps and GMRES tolerance")
    ap.add_argument("--instances", type=int, default=0,
                    help="batched workload: number of instances (0: 64); c4: training surfaces (0: 96)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0)
    ap.add_argument("--no-solve", action="store_true", help="skip the GMRES time-to-tolerance comparison")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--maxit", type=int, default=200, help="GMRES iteration limit (no restart below it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--coupling", type=float, default=-1.0,
                    help="Burton-Miller alpha = i*coupling/k; 1 is the value the paper states, -1 its conjugate")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        return 2
    import numpy as np
    import torch

    import paper_1311_5202_amd as fdb
    import synth

    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload in BATCH:
        return batch_main(args, fdb, synth, torch)
    if args.workload in LEARNED:
        return learned_main(args, fdb, synth, torch)
    if args.workload in RADIATION:
        return radiation_main(args, fdb, synth, torch)
    if args.workload in TABLE1:
        return table1_main(args, fdb, synth, torch)
    n_split, k, eps, desc = WORKLOADS[args.workload]
    aspect = ELONGATED.get(args.workload)
    el = synth.octa_sphere(n_split) if aspect is None else synth.ellipsoid(n_split, aspect)
    pts, nrm, w = fdb.nystrom_nodes(el)
    N = len(w)
    t0 = time.perf_counter()
    plan = fdb.build(pts, nrm, w, k, eps, elements=el if aspect is None else None, corrections=1, verbose=1,
                     precision="both", coupling=args.coupling)
    t_build = time.perf_counter() - t0
    st = plan.stats()
    print(f"[bench] workload={args.workload} N={N} k={k} p2p_pairs={st['p2p_pairs']} build {t_build:.1f} s m2l_tile={st.get('m2l_tile')} tiles(t,ch,p,seg)={st.get('m2l_tiles')} lds={st.get('m2l_lds_bytes')}/{st.get('max_lds_per_block')}", file=sys.stderr, flush=True)
    u_host = synth.random_densities(N, 1)
    u = torch.from_numpy(u_host).cuda()
    out = torch.empty_like(u)
    op = "BM_H" if st.get("corr_nnz", 0) > 0 else "RAW_H"
    for _ in range(args.warmup):
        plan.matvec(u, op, out=out)
    torch.cuda.synchronize()
    # every step bracketed by HIP events on the stream the library launches on
    # (torch's current stream); the whole run by the host clock
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record()
        plan.matvec(u, op, out=out)
        e1.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step_ms = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    ms_median = step_ms[len(step_ms) // 2] if len(step_ms) % 2 else 0.5 * (
        step_ms[len(step_ms) // 2 - 1] + step_ms[len(step_ms) // 2])
    # per-phase HIP-event times over a second pass of the same steps
    plan.set_timing(True)
    for _ in range(args.steps):
        plan.matvec(u, op, out=out)
    phases = plan.phase_times()
    plan.set_timing(False)
    torch.cuda.synchronize()
    # FP32 far and near field on the same densities
    out32 = torch.empty_like(u)
    plan.matvec(u, op, out=out32, fp32=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.matvec(u, op, out=out32, fp32=True)
    torch.cuda.synchronize()
    dt32 = time.perf_counter() - t0
    # the FP32 error on the uncorrected H sum, where no FP64 term dilutes it
    raw64 = plan.matvec(u, "RAW_H")
    raw32 = plan.matvec(u, "RAW_H", fp32=True)
    fp32 = {"matvec_per_s": args.steps / dt32,
            "rel_l2_vs_fp64": (torch.linalg.norm(out32 - out) / torch.linalg.norm(out)).item(),
            "raw_h_rel_l2_vs_fp64": (torch.linalg.norm(raw32 - raw64) / torch.linalg.norm(raw64)).item()}
    del raw64, raw32
    print(f"[bench] FP32 mat-vec {fp32}", file=sys.stderr, flush=True)
    ms = ms_median
    free, total = torch.cuda.mem_get_info()
    peak_used = total - free
    flops, byts = m2l_work(st)
    m2l_ms = phases["m2l"]
    # kernel launches in the M2L phase: per slab one chunk kernel and one segmented sum
    n_m2l_launch = max(1, 2 * sum(t[0] for t in st.get("m2l_tiles", []) if t[0] > 0)) if st.get("m2l_mode") == 3 \
        else max(1, sum(1 for L in st["levels"] if L["m2l_pairs"] > 0))
    roof = {
        "bound": "mfma",
        "kernel": "M2L (all levels of one mat-vec)",
        "achieved": flops / (m2l_ms * 1e-3) / 1e12 if m2l_ms > 0 else 0.0,
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "traffic": measured_traffic(args.workload),
        "launches_per_matvec": n_m2l_launch,
        "algorithmic_flops_per_matvec": flops,
        "algorithmic_bytes_per_matvec": byts,
    }
    roof["frac"] = roof["achieved"] / roof["peak"]
    # P2P against the FP64 vector peak (operation count per pair above)
    p2p_flops = P2P_FLOPS_PER_PAIR * st["p2p_pairs"]
    p2p_roof = {"bound": "valu", "kernel": "P2P (near-field point sums)",
                "achieved": p2p_flops / (phases["p2p"] * 1e-3) / 1e12 if phases["p2p"] > 0 else 0.0,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "flops_per_pair": P2P_FLOPS_PER_PAIR,
                "pairs": st["p2p_pairs"],
                "pairs_per_s": st["p2p_pairs"] / (phases["p2p"] * 1e-3) if phases["p2p"] > 0 else 0.0}
    p2p_roof["frac"] = p2p_roof["achieved"] / p2p_roof["peak"]
    res = {
        "metric": "FDA matvecs/s (Burton-Miller H operator)",
        "value": args.steps / dt,
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_mean": 1e3 * dt / args.steps,
        "ms_per_step_min_max": [step_ms[0], step_ms[-1]],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "N": N, "k": k, "eps": eps, "operator": op,
                   "alpha": f"{args.coupling:g}i/k", "parallelism": "single GPU"},
        "phase_ms": phases,
        "build_s": t_build,
        "roofline": roof,
        "p2p_roofline": p2p_roof,
        "phase_rooflines": phase_rooflines(st, phases),
        "fp32": fp32,
    }
    if not args.no_solve and op == "BM_H":
        log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
        res["gmres"] = gmres_compare(fdb, synth, plan, 1e-4, args.coupling, args.epochs, log, args.maxit)
    free, total = torch.cuda.mem_get_info()
    res["peak_device_gb"] = max(peak_used, total - free) / 1e9
    res["plan_device_gb"] = plan.stats().get("device_bytes", 0) / 1e9
    if not args.no_cpu_baseline:
        n_rows = args.cpu_rows or max(64, min(N, int(2.5e9 / N)))
        # the same raw H sum on the GPU (FP64 and FP32) for parity on the oracle's sample
        raw = {"raw_h_fp64": plan.matvec(u, "RAW_H").cpu().numpy(),
               "raw_h_fp32": plan.matvec(u, "RAW_H", fp32=True).cpu().numpy()}
        res["cpu_baseline"] = cpu_baseline(pts, nrm, w, u_host, k, n_rows, raw, args.coupling)
    plan.close()
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
