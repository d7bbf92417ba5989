"""Benchmark of the H^2 matvec and GMRES time-to-1e-8 on one MI355X.

Workload: Laplace single layer on the unit sphere as 6 cube-sphere patches, level 6,
degree-2 B-splines (N = 26,136), H^2 with 5x5 Chebyshev points per cluster, eta = 1.6,
leaf level 4.  A step is one H^2 matvec y = A x (forward, upward, coupling, downward,
backward + near field) on a seeded random x resident in HBM, in FP64.

The headline is the faster of the two FP64 far-field variants: the coupling evaluated on
the fly from the clusters' Chebyshev points (bound by FP64 arithmetic), and the coupling
blocks stored at assembly (bound by HBM traffic), both reported with their roofline.
Prints one JSON line (metric, value = DOF/s, ...), the roofline of the dominant kernel
from HIP events around that stage, the GMRES solve to a relative residual of 1e-8, and the
CPU oracle timed on a bounded sample of the same workload.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gmres", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="skip the many-RHS Helmholtz workload")
    ap.add_argument("--no-c3", action="store_true", help="skip the batched uneven workload")
    ap.add_argument("--c3-instances", type=int, default=512)
    ap.add_argument("--no-c4", action="store_true", help="skip the learned-preconditioner workload")
    ap.add_argument("--tune", action="store_true", help="run the autotuner on the main workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--only-main", action="store_true", help="main workload matvec only (for profiling)")
    ap.add_argument("--only-c2", action="store_true", help="many-RHS Helmholtz matvecs only (for profiling)")
    ap.add_argument("--cpu-rows", type=int, default=24, help="sampled rows for the oracle's near-field timing")
    ap.add_argument("--no-cpu-legs", action="store_true", help="skip the oracle's timings of the other workloads")
    ap.add_argument("--no-maxwell", action="store_true", help="skip the Maxwell single-layer workload")
    ap.add_argument("--only-maxwell", action="store_true", help="Maxwell workload only")
    ap.add_argument("--maxwell-matvec-only", action="store_true",
                    help="Maxwell workload: assembly and matvec timings only (for profiling)")
    return ap.parse_args()


# FP64 operations per coupling entry evaluated on the fly, the method's own work (a fused
# multiply-add counts 2): squared distance of two points (3 differences, 3 products, 2
# sums = 8), one reciprocal square root (1), the entry's product with the moment in the row
# sum and in the transposed product (4) = 13.  The kernel issues 20: the squared distance
# expanded about the owner's first point (1 add + 3 FMA = 7), the hardware estimate (1) and
# its third-order correction (2 mul + 3 FMA = 8), the two products (4); that count is
# reported beside it.
OTF_FLOPS_PER_ENTRY = 13
OTF_ISSUED_FLOPS_PER_ENTRY = 20
FP64_VECTOR_PEAK_TFLOPS = 78.6


def measured_traffic(kernel="k_coupling"):
    """HBM bytes per launch of a kernel from the committed counter summary, if the kernel
    source is still the one the counters were taken with (else None)."""
    import hashlib
    import re

    src = os.path.join(ROOT, "paper_1906_00785_amd", "csrc", "bem_kernels.hip")
    md = os.path.join(ROOT, "profiles", f"{kernel}_laplace_sphere6_L6_d2_hbm_counters.md")
    if not os.path.exists(md):
        return None
    txt = open(md).read()
    h = re.search(r"kernel_source_sha256_16: ([0-9a-f]+)", txt)
    t = re.search(r"traffic_bytes_per_launch: ([0-9.]+)", txt)
    if not h or not t:
        return None
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return float(t.group(1)) if cur == h.group(1) else None


def _sampled_matvec_s(H, x, N, nrows, seed_cfg, reps=5):
    """Seconds of one oracle H^2 matvec: the far field (forward, upward, coupling, downward,
    backward) over all N rows timed in full, the near field over `nrows` seeded rows
    (assembled first, untimed) timed and scaled to N rows."""
    import numpy as np

    import workloads as W

    rows = W.sample_rows(seed_cfg, N, nrows)
    H.assemble_near_rows(rows)
    allrows = np.arange(N, dtype=np.int64)
    t0 = time.perf_counter()
    H.apply_rows(x, allrows, far=True, near=False)
    t_far = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(reps):
        H.apply_rows(x, rows, far=False, near=True)
    t_near = (time.perf_counter() - t0) / reps * (N / rows.size)
    return t_far, t_near, rows.size


def _cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


def cpu_baseline(cfg, x, nrows, threads=1):
    """Oracle H^2 matvec on the same workload (the oracle as it stands, plain FP64), timed on
    a bounded sample: far field over all rows in full, near field on sampled rows scaled to
    N rows.  threads > 1: the oracle's timing mode (parallel loops over independent rows,
    clusters and target runs; the same results)."""
    import oracle as O

    used = O.set_threads(threads)
    S = O.Space(O.SPHERE, [], O.LAPLACE, 0.0, degree=cfg["degree"], level=cfg["level"])
    H = O.H2(S, q=cfg["q"], eta=cfg["eta"], leaf=cfg["leaf"], qg=cfg["qg"], qs=cfg["qs"], assemble_near=False)
    N = S.ndof
    t_far, t_near, nr = _sampled_matvec_s(H, x, N, nrows, 1)
    t = t_far + t_near
    O.set_threads(1)
    return {"value": N / t, "unit": "DOF/s", "cores": used, "kind": "oracle",
            "sample": f"far field over all {N} rows timed in full ({t_far:.3f} s); near field timed over "
                      f"{nr} seeded rows and scaled to {N} rows ({t_near:.3f} s); FP64, {used} thread(s)"}


def cpu_oracle_legs(args, gpu):
    """The oracle on the other workloads, bounded samples on the host cores (timing mode with
    every core the process may use; the oracle's results do not depend on the thread count).
    gpu: the GPU figures the estimates are scaled with (iteration counts) or compared to."""
    import numpy as np

    import oracle as O
    import workloads as W

    model, ncpu = _cpu_info()
    used = O.set_threads(ncpu)
    out = {"cpu_model": model, "nproc": ncpu, "threads": used}
    # C0: dense assembly, solve and potential, in full
    c0 = W.CONFIGS[0]
    t0 = time.perf_counter()
    S0 = O.Space(O.SPHERE, [], O.LAPLACE, 0.0, degree=c0["degree"], level=c0["level"])
    A0 = S0.dense(c0["qg"], c0["qs"])
    t_asm = time.perf_counter() - t0
    x0, pts = W.c0_inputs()
    t0 = time.perf_counter()
    rho = np.linalg.solve(A0, S0.rhs(O.POINT_SOURCE, x0))
    u = S0.potential(rho, pts)
    t_sol = time.perf_counter() - t0
    ex = 1.0 / (4 * np.pi * np.linalg.norm(pts - np.array(x0), axis=1))
    out["c0_dense"] = {"assembly_s": t_asm, "solve_and_potential_s": t_sol,
                       "potential_max_rel_err": float(np.max(np.abs(u - ex)) / np.max(np.abs(ex))),
                       "sample": "in full"}
    # C1 GMRES: one sampled matvec times the GPU's iteration count (the Arnoldi steps' vector
    # work is small beside the matvec)
    c1 = W.CONFIGS[1]
    S1 = O.Space(O.SPHERE, [], O.LAPLACE, 0.0, degree=c1["degree"], level=c1["level"])
    H1 = O.H2(S1, q=c1["q"], eta=c1["eta"], leaf=c1["leaf"], assemble_near=False)
    x1 = W.random_vector(W.rng(1, 11), S1.ndof)
    tf, tn, nr = _sampled_matvec_s(H1, x1, S1.ndof, 24, 1, reps=3)
    its = gpu.get("c1_gmres_iterations")
    out["c1_gmres"] = {"matvec_s": tf + tn, "iterations": its,
                       "time_to_tol_s_estimate": (tf + tn) * its if its else None,
                       "sample": f"one matvec (far field in full, near field on {nr} rows scaled) times the GPU "
                                 f"solve's iteration count"}
    # C2: one wavenumber, one of the 128 columns, scaled to 128
    c2 = W.CONFIGS[2]
    kappa, dirs = W.c2_inputs()
    S2 = O.Space(O.SPHERE, [], O.HELMHOLTZ, kappa, degree=c2["degree"], level=c2["level"])
    t0 = time.perf_counter()
    H2 = O.H2(S2, q=c2["q"], eta=c2["eta"], leaf=c2["leaf"], assemble_near=False)
    t_far_asm = time.perf_counter() - t0
    x2 = W.random_vector(W.rng(2, 11), S2.ndof, is_complex=True)
    tf, tn, nr = _sampled_matvec_s(H2, x2, S2.ndof, 12, 2, reps=3)
    out["c2_many_rhs"] = {"far_assembly_s": t_far_asm, "matvec_one_column_s": tf + tn,
                          "dof_rhs_per_s": S2.ndof / (tf + tn),
                          "sample": f"one column (far field in full, near field on {nr} rows scaled); the "
                                    f"oracle applies columns one after the other, so 128 take 128 times as long"}
    # C3: 32 seeded instances, one column each timed, times their column counts
    insts = W.c3_instances(32)
    tot, dofrhs, tbuild = 0.0, 0, 0.0
    for k, it in enumerate(insts):
        S = O.Space(it["geom"], list(it["params"]), it["pde"], it["kappa"], degree=it["degree"], level=it["level"])
        t0 = time.perf_counter()
        H = O.H2(S, q=W.CONFIGS[3]["q"], eta=W.CONFIGS[3]["eta"], leaf=max(it["level"] - 2, 0), assemble_near=False)
        tbuild += time.perf_counter() - t0
        xx = W.random_vector(W.rng(3, 500 + k), S.ndof, is_complex=bool(it["pde"]))
        tf, tn, _ = _sampled_matvec_s(H, xx, S.ndof, 3, 3, reps=1)
        nc = len(it["sources"])
        tot += (tf + tn) * nc
        dofrhs += S.ndof * nc
    out["c3_subset"] = {"instances": len(insts), "dof_rhs": dofrhs, "matvec_s": tot, "dof_rhs_per_s": dofrhs / tot,
                        "far_assembly_s": tbuild,
                        "sample": "the first 32 seeded instances: one column each (far field in full, near field "
                                  "on 3 rows scaled), times its column count"}
    # C4: the correction network in FP64 (forward + loss gradient) on a 1,024-block batch
    import oracle.mlp as M

    g = W.rng(4, 900)
    nin, hid, nout = 99, 256, 2048
    P = g.normal(scale=0.05, size=M.nparams(nin, hid, nout))
    Xb = g.normal(size=(1024, nin))
    Tb = g.normal(size=(1024, 64, 64)) + 1j * g.normal(size=(1024, 64, 64))
    t0 = time.perf_counter()
    M.loss_and_grad(P, Xb, Tb, nin, hid, nout, True)
    t_mlp = time.perf_counter() - t0
    out["c4_network"] = {"blocks": 1024, "forward_and_gradient_s": t_mlp, "blocks_per_s": 1024 / t_mlp,
                         "sample": "numpy FP64 forward, rank-8 loss and gradient of the 99-256-256-2048 network"}
    O.set_threads(1)
    return out


BF16_MFMA_PEAK = 2.5e15


def bench_c2(B, W, torch, np, stream, args):
    """Helmholtz single layer, sphere level 5, degree 2, 128 plane waves: the many-RHS
    matvec (FP64, FP32 far field, BF16 far field on the matrix cores) and lockstep GMRES to
    1e-8 in FP64 and with FP64 refinement around the FP32 far field."""
    c = W.CONFIGS[2]
    kappa, dirs = W.c2_inputs()
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_HELMHOLTZ_SINGLE, kappa, degree=c["degree"], level=c["level"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A16 = B.Operator(s, q=c["q"], eta=c["eta"], leaf_level=c["leaf"], far_low=B.BEM_PREC_BF16, batch_rhs=c["nrhs"])
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    A32 = B.Operator(s, q=c["q"], eta=c["eta"], leaf_level=c["leaf"], far_low=B.BEM_PREC_FP32, batch_rhs=c["nrhs"])
    N, R, q2 = s.ndof, c["nrhs"], c["q"] ** 2
    info = A16.info
    b = s.rhs(B.BEM_DATA_PLANE_WAVE, dirs)
    y = torch.empty_like(b)
    steps = max(5, min(args.steps // 10, 30))
    out = {"workload": c["name"], "ndof": N, "nrhs": R, "kappa": kappa, "leaf_level": c["leaf"], "nfar": info.nfar,
           "near_nnz": info.near_nnz, "assembly_s": t_asm}
    for name, op, prec in (("fp64", A16, 0), ("fp32", A32, B.BEM_PREC_FP32), ("bf16", A16, B.BEM_PREC_BF16)):
        for _ in range(2):
            op.apply(b, out=y, prec=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            op.apply(b, out=y, prec=prec)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        op.profile(True)
        for _ in range(steps):
            op.apply(b, out=y, prec=prec)
        st_ms, _ = op.profile_read()
        op.profile(False)
        # useful far-field flops: every ordered block applied to every column (complex: 8 per entry)
        flops = info.nfar * q2 * q2 * 8.0 * R
        ent = {"matvec_ms": ms, "dof_rhs_per_s": N * R / (ms * 1e-3),
               "stages_ms": {"moments": st_ms[0], "coupling": st_ms[1], "down_back": st_ms[2], "near_out": st_ms[3]},
               "coupling_useful_tflops": flops / (st_ms[1] * 1e-3) / 1e12}
        if prec == B.BEM_PREC_BF16:
            ent["coupling_mfma_frac_of_bf16_peak"] = flops / (st_ms[1] * 1e-3) / BF16_MFMA_PEAK
        out[name] = ent
        print(f"bench c2: {name} matvec {ms:.3f} ms ({N*R/(ms*1e-3):.3e} DOF*RHS/s); stages "
              f"{st_ms[0]:.3f}/{st_ms[1]:.3f}/{st_ms[2]:.3f}/{st_ms[3]:.3f} ms; coupling "
              f"{flops/(st_ms[1]*1e-3)/1e12:.1f} TFLOP/s useful", file=sys.stderr, flush=True)
    if not args.no_gmres:
        A16.precond_build()
        A32.precond_build()
        for name, op, refine, pc in (("gmres_fp64", A16, False, False), ("gmres_fp32_refined", A32, True, False),
                                     ("gmres_bf16_refined", A16, True, False),
                                     ("gmres_fp64_block_jacobi", A16, False, True),
                                     ("gmres_fp32_refined_block_jacobi", A32, True, True),
                                     ("gmres_bf16_refined_block_jacobi", A16, True, True)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = op.solve(b, tol=c["tol"], restart=c["restart"], maxit=c["maxit"], refine=refine, precond=pc)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            its = [v[0] for v in st]
            res = float(((b - A16.apply(x)).norm(dim=1) / b.norm(dim=1)).max())
            out[name] = {"time_to_tol_s": t, "iterations_min": min(its), "iterations_max": max(its),
                         "converged": sum(bool(v[1]) for v in st), "max_true_relres": res,
                         "outer_max": max(v[3] for v in st)}
            base = "gmres_fp64_block_jacobi" if pc else "gmres_fp64"
            if name != base:
                out[name]["speedup_vs_fp64"] = out[base]["time_to_tol_s"] / t
            print(f"bench c2: {name} {t:.3f}s its {min(its)}..{max(its)} converged {out[name]['converged']}/{R} "
                  f"max relres {res:.2e}", file=sys.stderr, flush=True)
        # the stated error of the refined solutions: all to 1e-12, max over the 128 columns of
        # the relative difference to the FP64 solution
        x64, _ = A16.solve(b, tol=1e-12, restart=c["restart"], maxit=20000)
        for name, op in (("gmres_fp32_refined", A32), ("gmres_bf16_refined", A16)):
            xl, _ = op.solve(b, tol=1e-12, restart=c["restart"], maxit=20000, refine=True, max_outer=40)
            err = float(((xl - x64).norm(dim=1) / x64.norm(dim=1)).max())
            out[name]["solution_rel_err_vs_fp64_at_1e-12"] = err
            print(f"bench c2: {name} solution error vs FP64 (all to 1e-12) {err:.1e}", file=sys.stderr, flush=True)
    return out


def dipole_field(prm, kappa, pts, np):
    """Field of the electric dipole (moment m at x0) at the points, closed form:
    E = kappa^2 G m + g'(r) (m . R) R / r + g(r) m with G = exp(-i kappa r) / (4 pi r) and
    g = G' / r (the curl curl of m G)."""
    x0, m = np.asarray(prm[:3]), np.asarray(prm[3:])
    R = pts - x0
    r = np.linalg.norm(R, axis=1)[:, None]
    ik = 1j * kappa
    ex = np.exp(-ik * r) / (4 * np.pi)
    G = ex / r
    G1 = -ex * (1 + ik * r) / r ** 2
    G2 = ex * (2 + 2 * ik * r + (ik * r) ** 2) / r ** 3
    gg, gp = G1 / r, (G2 - G1 / r) / r
    return kappa ** 2 * G * m + gp * (R @ m)[:, None] * R / r + gg * m


def bench_maxwell(B, W, torch, np, stream, args):
    """Maxwell single layer (EFIE) on the unit sphere, dipole data: compressed operator at
    the workload level (plan, assembly, matvec by HIP events, GMRES to 1e-8, field error at
    exterior points), the dense operator's matvec at a small level, the field error over the
    levels at degrees 1 and 2 (the paper's Fig. 1 series), and the oracle's compressed
    assembly timed on the host beside the GPU's at a small level."""
    c = W.MAXWELL
    prm, pts = W.maxwell_inputs()
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    exact = dipole_field(prm, c["kappa"], pts, np)
    out = {"workload": c["name"], "kappa": c["kappa"], "q": c["q"], "eta": c["eta"]}

    def field_err(s, x):
        E = s.potential(pts, x).cpu().numpy()
        return float(np.abs(E - exact).max() / np.abs(exact).max())

    steps = max(5, min(args.steps // 4, 50))
    for leaf_off in (1, 0):
        s = B.Space(g, B.BEM_MAXWELL_SINGLE, c["kappa"], degree=c["degree"], level=c["level"])
        leaf = c["level"] - leaf_off
        t0 = time.perf_counter()
        A = B.Operator(s, q=c["q"], eta=c["eta"], leaf_level=leaf, qg=c["qg"], qs=c["qs"], assemble=False)
        t_plan = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A.assemble()
        torch.cuda.synchronize()
        t_asm = time.perf_counter() - t0
        N, info = A.ndof, A.info
        x = torch.from_numpy(W.random_vector(W.rng(14, N), N, True)).cuda()
        y = torch.empty_like(x)
        for _ in range(3):
            A.apply(x, out=y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            A.apply(x, out=y)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        nl, q2 = 2 * c["degree"] * (c["degree"] + 1), c["q"] ** 2
        nelem = 6 * 4 ** c["level"]
        # bytes every apply must move: kernel blocks (one per admissible pair), near blocks,
        # channel moments (read in the forward and the backward transform), and the blocks'
        # transposed products (written by the coupling, read by the top-down pass)
        byts = info.far_bytes + info.near_bytes + 2.0 * nelem * nl * 4 * q2 * 8 + 2.0 * info.nstored * 4 * q2 * 16
        ent = {"leaf_level": leaf, "ndof": N, "nfar": info.nfar, "nstored": info.nstored, "near_leaf_pairs": info.nnear,
               "near_block_entries": info.near_nnz, "far_bytes": info.far_bytes, "near_bytes": info.near_bytes,
               "plan_s": t_plan, "assembly_s": t_asm, "matvec_ms": ms, "dof_per_s": N / (ms * 1e-3),
               "matvec_gbs": byts / (ms * 1e-3) / 1e9}
        print(f"bench maxwell: leaf {leaf} N={N} far={info.nfar} near={info.nnear} plan {t_plan:.2f}s assemble "
              f"{t_asm:.3f}s matvec {ms:.3f} ms ({N/(ms*1e-3):.3e} DOF/s, {ent['matvec_gbs']:.0f} GB/s of "
              f"{byts/1e9:.2f} GB)", file=sys.stderr, flush=True)
        if leaf_off == 1 and not args.no_gmres:
            b = s.rhs(B.BEM_DATA_DIPOLE, [prm])[0]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sol, st = A.solve(b, tol=c["tol"], restart=c["restart"], maxit=c["maxit"])
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            rr = float((b - A.apply(sol)).norm() / b.norm())
            ent["gmres"] = {"time_to_tol_s": t, "iterations": st[0][0], "converged": bool(st[0][1]), "relres": rr,
                            "field_rel_err": field_err(s, sol)}
            print(f"bench maxwell: GMRES({c['restart']}) {st[0][0]} its {t:.3f}s relres {rr:.2e} field error "
                  f"{ent['gmres']['field_rel_err']:.2e}", file=sys.stderr, flush=True)
        out[f"leaf_L-{leaf_off}"] = ent
        del A
    if args.maxwell_matvec_only:
        return out
    # dense operator at a small level: the matvec reads N^2 complex entries
    Ld = c["dense_level"]
    s = B.Space(g, B.BEM_MAXWELL_SINGLE, c["kappa"], degree=c["degree"], level=Ld)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ad = B.Operator(s, eta=0.0, qg=c["qg"], qs=c["qs"])
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    N = Ad.ndof
    x = torch.from_numpy(W.random_vector(W.rng(14, N), N, True)).cuda()
    y = torch.empty_like(x)
    for _ in range(3):
        Ad.apply(x, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        Ad.apply(x, out=y)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    out["dense"] = {"level": Ld, "ndof": N, "assembly_s": t_asm, "matvec_ms": ms,
                    "matvec_gbs": N * N * 16 / (ms * 1e-3) / 1e9}
    print(f"bench maxwell: dense L{Ld} N={N} assemble {t_asm:.3f}s matvec {ms:.4f} ms "
          f"({out['dense']['matvec_gbs']:.0f} GB/s of the matrix)", file=sys.stderr, flush=True)
    del Ad
    # field error over the levels (compressed operator, leaf L - 1), degrees 1 and 2
    series = {}
    for p in (1, 2):
        errs, its, res = [], [], []
        for L in c["levels"]:
            s = B.Space(g, B.BEM_MAXWELL_SINGLE, c["kappa"], degree=p, level=L)
            A = B.Operator(s, q=c["series_q"], eta=c["eta"], leaf_level=max(L - 1, 0), qg=c["qg"], qs=c["qs"])
            b = s.rhs(B.BEM_DATA_DIPOLE, [prm])[0]
            sol, st = A.solve(b, tol=c["series_tol"], restart=c["restart"], maxit=c["series_maxit"])
            errs.append(field_err(s, sol))
            its.append(st[0][0])
            res.append(st[0][2])
            del A
        eoc = [float(np.log2(errs[k] / errs[k + 1])) for k in range(len(errs) - 1)]
        series[f"p{p}"] = {"levels": list(c["levels"]), "q": c["series_q"], "field_rel_err": errs, "eoc": eoc,
                           "gmres_iterations": its, "gmres_relres": res}
        print(f"bench maxwell: p = {p} (q = {c['series_q']}) field errors {['%.2e' % e for e in errs]} orders "
              f"{['%.2f' % v for v in eoc]} GMRES its {its} relres {['%.1e' % v for v in res]}", file=sys.stderr,
              flush=True)
    out["convergence"] = series
    if not args.no_cpu_baseline:
        # cpu-baseline leg: the oracle's compressed matrix (host, all cores) beside the GPU's
        # assembly + N matvecs
        import oracle

        Lc = 2
        So = oracle.MSpace(oracle.SPHERE, [], c["kappa"], p=c["degree"], level=Lc)
        t0 = time.perf_counter()
        So.h2_dense(q=c["q"], eta=c["eta"], leaf=Lc - 1, qg=c["qg"], qs=c["qs"])
        t_orc = time.perf_counter() - t0
        s = B.Space(g, B.BEM_MAXWELL_SINGLE, c["kappa"], degree=c["degree"], level=Lc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A = B.Operator(s, q=c["q"], eta=c["eta"], leaf_level=Lc - 1, qg=c["qg"], qs=c["qs"])
        A.apply(torch.eye(A.ndof, dtype=torch.complex128, device="cuda"))
        torch.cuda.synchronize()
        t_gpu = time.perf_counter() - t0
        out["cpu_oracle"] = {"kind": "oracle", "sample": f"compressed matrix, sphere L{Lc} p{c['degree']}",
                             "ndof": A.ndof, "oracle_s": t_orc, "gpu_assembly_and_columns_s": t_gpu}
        print(f"bench maxwell: oracle compressed matrix L{Lc} {t_orc:.2f}s, GPU assembly + {A.ndof} columns "
              f"{t_gpu:.3f}s", file=sys.stderr, flush=True)
    return out


def bench_c3(B, W, torch, np, args):
    """Batched uneven instances, every instance and right-hand side in FP64: per-column
    applies, one grouped launch per stage over every instance and column, and the grouped
    launches captured into one graph.  Laplace instances evaluate the coupling on the fly,
    Helmholtz instances stream their stored blocks (measured faster in grouped launches,
    where an operator's columns read them one after the other)."""
    import paper_1906_00785_amd.autotune as AT

    insts = W.c3_instances(args.c3_instances)
    q3, eta3 = W.CONFIGS[3]["q"], W.CONFIGS[3]["eta"]
    # autotuned launch shapes (leaf level, coupling chunk width) per shape class of the two
    # largest levels, measured on the class's first instance and used for all of its members
    t0 = time.perf_counter()
    tuned = {}
    for it in insts:
        cls = (it["geom"], it["pde"], it["level"], it["degree"])
        if it["level"] < 4 or cls in tuned:
            continue
        g = B.Geometry(it["geom"], it["params"])
        s = B.Space(g, it["pde"], it["kappa"], degree=it["degree"], level=it["level"])
        r = AT.tune(s, q=q3, eta=eta3, steps=5, far_eval=it["pde"] == 0,
                    leaf_levels=[lv for lv in (it["level"] - 3, it["level"] - 2, it["level"] - 1) if lv >= 0])
        tuned[cls] = {"leaf_level": r["leaf_level"], "chunk_cols": r["chunk_cols"], "apply_us": r["apply_us"]}
        del s, g
    t_tune = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    members = {0: [], 1: []}
    for it in insts:
        g = B.Geometry(it["geom"], it["params"])
        s = B.Space(g, it["pde"], it["kappa"], degree=it["degree"], level=it["level"])
        tc = tuned.get((it["geom"], it["pde"], it["level"], it["degree"]))
        A = B.Operator(s, q=q3, eta=eta3, leaf_level=tc["leaf_level"] if tc else max(it["level"] - 2, 0),
                       chunk_cols=tc["chunk_cols"] if tc else 0, far_eval=it["pde"] == 0)
        x = s.rhs(B.BEM_DATA_POINT_SOURCE, it["sources"])
        members[it["pde"]].append((s, A, x, torch.empty_like(x)))
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    dofrhs = sum(s.ndof * x.shape[0] for m in members.values() for s, _, x, _ in m)
    groups = [B.Group([A for _, A, _, _ in m], [x for _, _, x, _ in m], [y for _, _, _, y in m])
              for m in members.values() if m]
    side = torch.cuda.Stream()
    reps = 5

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def per_column():
        for m in members.values():
            for s, A, x, y in m:
                A.apply(x, out=y)

    def grouped():
        for G in groups:
            G.apply()

    t_col = timed(per_column)
    t_group = timed(grouped)
    with torch.cuda.stream(side):
        graph = B.Graph()
        with graph:
            grouped()
        t_graph = timed(graph.launch)
    torch.cuda.synchronize()
    nrhs = sum(x.shape[0] for m in members.values() for _, _, x, _ in m)
    out = {"workload": W.CONFIGS[3]["name"], "instances": len(insts), "columns": nrhs, "dof_rhs": dofrhs,
           "assembly_s": t_asm, "per_column_ms": t_col, "grouped_ms": t_group, "graph_ms": t_graph,
           "dof_rhs_per_s_graph": dofrhs / (t_graph * 1e-3), "dof_rhs_per_s_per_column": dofrhs / (t_col * 1e-3),
           "far_field": "on the fly (Laplace), stored blocks (Helmholtz)", "launches_grouped": 6 * len(groups),
           "autotune_s": t_tune,
           "autotuned": {f"geom{k[0]}_pde{k[1]}_L{k[2]}_d{k[3]}": v for k, v in tuned.items()}}
    print(f"bench c3: {len(insts)} instances, {nrhs} columns, {dofrhs} DOF*RHS; assembly {t_asm:.1f}s; matvec "
          f"per-column {t_col:.2f} ms, grouped {t_group:.2f} ms, graph {t_graph:.2f} ms "
          f"({dofrhs/(t_graph*1e-3):.3e} DOF*RHS/s)", file=sys.stderr, flush=True)
    return out


def bench_c4(B, W, torch, np, args):
    """Learned block-Jacobi correction on the family as configured: ellipsoids and tori,
    levels 5 and 6, degree 2, Helmholtz with wavenumbers 4..20; the BF16 network (3 layers
    of width 256) is trained on solver-generated targets of about 10,000 tiles, then GMRES to
    1e-8 runs on held-out instances without a preconditioner, with plain block-Jacobi and
    with the learned correction (kept only if it wins its selection cycle)."""
    import paper_1906_00785_amd.learned as L

    cfg = W.CONFIGS[4]

    def op_of(inst, level):
        geom, prm, kappa = inst
        g = B.Geometry(geom, prm)
        s = B.Space(g, B.BEM_HELMHOLTZ_SINGLE, kappa, degree=cfg["degree"], level=level)
        A = B.Operator(s, q=cfg["q"], eta=cfg["eta"], leaf_level=level - 2)
        A.precond_build()
        return s, A

    t0 = time.perf_counter()
    feats, targs, ntr, used = [], [], 0, []
    nmax = 40
    for inst, level in zip(W.c4_instances(nmax, stream=0), W.c4_levels(nmax, stream=0)):
        s, A = op_of(inst, level)
        f, t = L.training_data(A, ring=cfg["ring"])
        feats.append(f)
        targs.append(t)
        ntr += f.shape[0]
        used.append(level)
        del A, s
        if ntr >= cfg["train_blocks"]:
            break
    X, T = torch.cat(feats), torch.cat(targs)
    del feats, targs
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    print(f"bench c4: {X.shape[0]} training blocks from {len(used)} instances (levels {sorted(set(used))}) "
          f"in {t_data:.1f}s", file=sys.stderr, flush=True)
    net = L.CorrectionNet(cplx=True, hidden=256, seed=1906, precision=1)
    t0 = time.perf_counter()
    losses = net.train(X, T, steps=600, batch=64, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    rows = []
    for inst, level in zip(W.c4_instances(4, stream=1), W.c4_levels(4, stream=1)):
        s, A = op_of(inst, level)
        b = s.rhs(B.BEM_DATA_PLANE_WAVE, W.unit_vectors(W.rng(4, 103), 1))
        res = {}
        for name, pc in (("none", False), ("block_jacobi", True)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, st = A.solve(b, tol=cfg["tol"], restart=cfg["restart"], maxit=cfg["maxit"], precond=pc)
            torch.cuda.synchronize()
            res[name] = {"iterations": st[0][0], "time_s": time.perf_counter() - t1, "converged": st[0][1],
                         "relres": st[0][2]}
        t1 = time.perf_counter()
        kept, rr = L.install(A, net, b, restart=cfg["restart"])
        _, st = A.solve(b, tol=cfg["tol"], restart=cfg["restart"], maxit=cfg["maxit"], precond=True)
        torch.cuda.synchronize()
        res["learned"] = {"iterations": st[0][0], "time_s": time.perf_counter() - t1, "converged": st[0][1],
                          "relres": st[0][2], "kept": kept, "cycle_relres_plain_learned": rr}
        rows.append({"instance": [inst[0], list(inst[1]), inst[2]], "level": level, "ndof": s.ndof, **res})
        print(f"bench c4: L{level} {inst}: " + ", ".join(
            f"{k} {res[k]['iterations']} its {res[k]['time_s']:.2f}s relres {res[k]['relres']:.1e}"
            for k in ("none", "block_jacobi", "learned")) + f" (learned kept {kept})", file=sys.stderr, flush=True)
        del A, s
    return {"workload": cfg["name"], "levels": sorted(set(used)), "kappa_range": list(cfg["kappa_range"]),
            "train_blocks": int(X.shape[0]), "train_instances": len(used), "data_s": t_data, "train_s": t_train,
            "train_steps": 600, "network": "3 layers, width 256, BF16 products",
            "loss_first": float(np.mean(losses[:10])), "loss_last": float(np.mean(losses[-10:])), "held_out": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1906_00785_amd as B
    import workloads as W

    cfg = W.CONFIGS[1]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.only_c2:
        args.no_gmres = True
        print(json.dumps({"many_rhs": bench_c2(B, W, torch, np, stream, args)}))
        return
    if args.only_maxwell:
        print(json.dumps({"maxwell": bench_maxwell(B, W, torch, np, stream, args)}))
        return
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=cfg["degree"], level=cfg["level"])
    t0 = time.perf_counter()
    A = B.Operator(s, q=cfg["q"], eta=cfg["eta"], leaf_level=cfg["leaf"], qg=cfg["qg"], qs=cfg["qs"], assemble=False,
                   far_low=B.BEM_PREC_FP32)
    t_plan = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A.assemble()
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    info = A.info
    N = A.ndof
    print(f"bench: N={N} far={info.nfar} near_leaf_pairs={info.nnear} nnz={info.near_nnz} "
          f"plan {t_plan:.2f}s assemble {t_asm:.3f}s", file=sys.stderr, flush=True)

    x_host = W.random_vector(W.rng(1, 11), N)
    x = torch.from_numpy(x_host).cuda()
    y = torch.empty_like(x)

    def timed_steps(op):
        for _ in range(args.warmup):
            op.apply(x, out=y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            op.apply(x, out=y)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / args.steps
        # stage timing with HIP events on the same stream (same number of steps)
        op.profile(True)
        for _ in range(args.steps):
            op.apply(x, out=y)
        st, _ = op.profile_read()
        op.profile(False)
        # the coupling kernel alone: back-to-back launches of stage 1 after a full apply
        # (idempotent), without the launch gaps inside the stage events above
        op.apply(x, out=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            op.apply_stage(1, x, y)
        e1.record(stream)
        torch.cuda.synchronize()
        return t, st, e0.elapsed_time(e1) / args.steps

    q2 = cfg["q"] ** 2
    # stored coupling blocks: algorithmic bytes of one coupling launch are the stored blocks
    # (each admissible pair once), the transposed products written per stored column, the
    # chunk row sums, the partner indices and the moments read once
    ms_st, stage_st, kern_st = timed_steps(A)
    coupling_bytes = (info.far_bytes + info.transposed_bytes + info.nchunks * q2 * 8 + info.nstored * 4
                      + info.nclusters * q2 * 8)
    achieved_st = coupling_bytes / (kern_st * 1e-3) / 1e9
    near_bytes = info.near_nnz * 12 + (N + 1) * 8 + 2 * N * 8
    print(f"bench: stored-block matvec {ms_st*1e3:.1f} us; stages near+up {stage_st[0]*1e3:.1f} coupling "
          f"{stage_st[1]*1e3:.1f} gather+down {stage_st[2]*1e3:.1f} back {stage_st[3]*1e3:.1f} us; coupling "
          f"kernel {kern_st*1e3:.1f} us {achieved_st:.0f} GB/s; near {near_bytes/(stage_st[0]*1e-3)/1e9:.0f} GB/s",
          file=sys.stderr, flush=True)

    # coupling evaluated on the fly (no stored blocks): bound by FP64 arithmetic; the
    # algorithmic work is OTF_FLOPS_PER_ENTRY per entry of every stored pair's block
    t0 = time.perf_counter()
    Aot = B.Operator(s, q=cfg["q"], eta=cfg["eta"], leaf_level=cfg["leaf"], qg=cfg["qg"], qs=cfg["qs"],
                     far_eval=True)
    torch.cuda.synchronize()
    t_asm_ot = time.perf_counter() - t0
    ms_ot, stage_ot, kern_ot = timed_steps(Aot)
    entries = info.nstored * q2 * q2
    otf_tflops = OTF_FLOPS_PER_ENTRY * entries / (kern_ot * 1e-3) / 1e12
    print(f"bench: on-the-fly matvec {ms_ot*1e3:.1f} us; stages near+up {stage_ot[0]*1e3:.1f} coupling "
          f"{stage_ot[1]*1e3:.1f} gather+down {stage_ot[2]*1e3:.1f} back {stage_ot[3]*1e3:.1f} us; coupling "
          f"{otf_tflops:.1f} TFLOP/s FP64 ({entries / (kern_ot * 1e-3) / 1e12:.2f} T entries/s; kernel {kern_ot*1e3:.1f} us)",
          file=sys.stderr, flush=True)
    roof_st = {"bound": "hbm", "kernel": "k_coupling (far-field coupling, stored blocks)", "achieved": achieved_st,
               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved_st / HBM_PEAK_GBS,
               "traffic": measured_traffic("k_coupling"), "algorithmic_bytes": coupling_bytes,
               "avg_ms": kern_st, "stage_ms": stage_st[1]}
    roof_ot = {"bound": "alu", "kernel": "k_coupling_otf (far-field coupling evaluated on the fly, FP64 vector)",
               "achieved": otf_tflops, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": otf_tflops / FP64_VECTOR_PEAK_TFLOPS, "traffic": measured_traffic("k_coupling_otf"),
               "algorithmic_flops": OTF_FLOPS_PER_ENTRY * entries, "entries": entries, "avg_ms": kern_ot,
               "stage_ms": stage_ot[1], "issued_flops_per_entry": OTF_ISSUED_FLOPS_PER_ENTRY,
               "issued_tflops": OTF_ISSUED_FLOPS_PER_ENTRY * entries / (kern_ot * 1e-3) / 1e12,
               "issued_frac": OTF_ISSUED_FLOPS_PER_ENTRY * entries / (kern_ot * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS}
    if ms_ot <= ms_st:
        ms, stage_ms, roof, roof_other, head = ms_ot, stage_ot, roof_ot, roof_st, "on_the_fly"
    else:
        ms, stage_ms, roof, roof_other, head = ms_st, stage_st, roof_st, roof_ot, "stored_blocks"
    value = N / (ms * 1e-3)
    Ah = Aot if head == "on_the_fly" else A

    def time_apply(op, prec, steps):
        for _ in range(3):
            op.apply(x, out=y, prec=prec)
        torch.cuda.synchronize()
        a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            op.apply(x, out=y, prec=prec)
        b_.record(stream)
        torch.cuda.synchronize()
        t = a.elapsed_time(b_) / steps
        op.profile(True)
        for _ in range(steps):
            op.apply(x, out=y, prec=prec)
        st_ms, _ = op.profile_read()
        op.profile(False)
        return t, st_ms

    extra = {}
    # plain device copy of 1 GiB (read + write): the attainable streaming bandwidth
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 / (c0.elapsed_time(c1) / 10 * 1e-3) / 1e9
    del src, dst
    roof_st["frac_of_copy"] = achieved_st / copy_gbs
    extra["copy_gbs"] = copy_gbs
    print(f"bench: 1 GiB device copy {copy_gbs:.0f} GB/s; stored-block coupling at {achieved_st / copy_gbs:.2f} of it",
          file=sys.stderr, flush=True)
    # MALL-cold figures: before every timed launch a 1 GiB copy (4x the 256 MB last-level
    # cache) evicts the operator's data, so the launch streams its bytes from HBM; the
    # back-to-back figures above may partly hit in that cache
    flush_src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(2.0)
    flush_dst = torch.empty_like(flush_src)

    def cold_ms(fn, reps=10):
        fn()
        tot = 0.0
        for _ in range(reps):
            flush_dst.copy_(flush_src)
            a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b_.record(stream)
            torch.cuda.synchronize()
            tot += a.elapsed_time(b_)
        return tot / reps

    A.apply(x, out=y)
    cold_cpl = cold_ms(lambda: A.apply_stage(1, x, y))
    cold_near = cold_ms(lambda: A.apply_stage(0, x, y))
    cold_st = cold_ms(lambda: A.apply(x, out=y))
    cold_ot = cold_ms(lambda: Aot.apply(x, out=y))
    del flush_src, flush_dst
    extra["mall_cold"] = {
        "stored_coupling_kernel_ms": cold_cpl, "stored_coupling_gbs": coupling_bytes / (cold_cpl * 1e-3) / 1e9,
        "near_and_up_stage_ms": cold_near, "near_gbs": near_bytes / (cold_near * 1e-3) / 1e9,
        "matvec_stored_ms": cold_st, "matvec_on_the_fly_ms": cold_ot,
        "dof_per_s_on_the_fly": N / (cold_ot * 1e-3), "dof_per_s_stored": N / (cold_st * 1e-3),
        "flush": "1 GiB device copy before every timed launch"}
    print(f"bench: MALL-cold: stored coupling {cold_cpl*1e3:.1f} us ({coupling_bytes/(cold_cpl*1e-3)/1e9:.0f} GB/s), "
          f"near+up stage {cold_near*1e3:.1f} us ({near_bytes/(cold_near*1e-3)/1e9:.0f} GB/s), matvec stored "
          f"{cold_st*1e3:.1f} us, on the fly {cold_ot*1e3:.1f} us", file=sys.stderr, flush=True)
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        extra["copy_calibration_bytes"] = src.numel() * 8
        del src, dst
    if args.only_main:
        args.no_gmres = args.no_c2 = args.no_c3 = args.no_c4 = args.no_maxwell = True
        args.no_cpu_baseline = True
    # mixed precision: FP32 and BF16 copies of the coupling blocks (FP32 accumulation)
    A16 = None if args.only_main else B.Operator(s, q=cfg["q"], eta=cfg["eta"], leaf_level=cfg["leaf"], qg=cfg["qg"],
                                                  qs=cfg["qs"], far_low=B.BEM_PREC_BF16)
    mixed = {}
    for name, op, prec in (() if args.only_main else (("fp32", A, B.BEM_PREC_FP32), ("bf16", A16, B.BEM_PREC_BF16))):
        t, st_ms = time_apply(op, prec, args.steps)
        low_bytes = info.far_bytes / 8 * (4 if prec == B.BEM_PREC_FP32 else 2)
        cb = low_bytes + info.transposed_bytes + info.nchunks * q2 * 8 + info.nstored * 4 + info.nclusters * q2 * 8
        mixed[name] = {"matvec_us": t * 1e3, "dof_per_s": N / (t * 1e-3), "coupling_us": st_ms[1] * 1e3,
                       "coupling_gbs": cb / (st_ms[1] * 1e-3) / 1e9}
        print(f"bench: {name} matvec {t*1e3:.1f} us, coupling {st_ms[1]*1e3:.1f} us "
              f"({cb/(st_ms[1]*1e-3)/1e9:.0f} GB/s)", file=sys.stderr, flush=True)
    if not args.no_gmres:
        x0 = cfg["x0"]
        b = s.rhs(B.BEM_DATA_POINT_SOURCE, [x0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho, stats = Ah.solve(b, tol=cfg["tol"], restart=cfg["restart"], maxit=cfg["maxit"])
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        it, ok, rr, _ = stats[0]
        _, pts = W.c1_inputs()
        u = s.potential(pts, rho[0]).cpu().numpy()
        ex = 1.0 / (4 * np.pi * np.linalg.norm(pts - np.array(x0), axis=1))
        perr = float(np.max(np.abs(u - ex)) / np.max(np.abs(ex)))
        extra["gmres"] = {"time_to_tol_s": t_solve, "iterations": it, "converged": ok, "relres": rr,
                          "tol": cfg["tol"], "restart": cfg["restart"], "potential_max_rel_err": perr,
                          "far_field": head}
        if head == "on_the_fly":
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sts = A.solve(b, tol=cfg["tol"], restart=cfg["restart"], maxit=cfg["maxit"])
            torch.cuda.synchronize()
            extra["gmres_stored_blocks"] = {"time_to_tol_s": time.perf_counter() - t0, "iterations": sts[0][0],
                                            "converged": sts[0][1], "relres": sts[0][2]}
        # block-Jacobi right preconditioning (build included in the time)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ah.precond_build()
        rho_p, stp = Ah.solve(b, tol=cfg["tol"], restart=cfg["restart"], maxit=cfg["maxit"], precond=True)
        torch.cuda.synchronize()
        t_p = time.perf_counter() - t0
        rr_true = float(((b[0] - Ah.apply(rho_p[0])).norm() / b[0].norm()))
        extra["gmres_block_jacobi"] = {"time_to_tol_s": t_p, "iterations": stp[0][0], "converged": stp[0][1],
                                       "relres": rr_true}
        print(f"bench: block-Jacobi GMRES {stp[0][0]} its {t_p:.3f}s (build included) relres {rr_true:.2e}",
              file=sys.stderr, flush=True)
        print(f"bench: GMRES {it} its {t_solve:.3f}s relres {rr:.2e} potential err {perr:.2e}", file=sys.stderr,
              flush=True)
        # the stated error of the refined solutions (reading A20): every solve to 1e-13, the
        # refined solution against the FP64 one (whose matvec the parity tests pin)
        x64t, _ = A.solve(b, tol=1e-13, restart=cfg["restart"], maxit=20000)
        for name, op in (("fp32", A), ("bf16", A16)):
            for pc in (False, True):
                if pc:
                    op.precond_build()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xm, stm = op.solve(b, tol=cfg["tol"], restart=cfg["restart"], maxit=cfg["maxit"], refine=True,
                                   precond=pc)
                torch.cuda.synchronize()
                tm = time.perf_counter() - t0
                itm, okm, rrm, outm = stm[0]
                key = name if not pc else name + "_block_jacobi"
                ent = mixed.setdefault(key, {})
                ent.update({"time_to_tol_s": tm, "iterations": itm, "outer": outm, "converged": okm, "relres": rrm})
                if not pc:
                    xt, _ = op.solve(b, tol=1e-13, restart=cfg["restart"], maxit=20000, refine=True, max_outer=40)
                    ent["solution_rel_err_vs_fp64_at_1e-13"] = float((xt - x64t).norm() / x64t.norm())
                ent["speedup_vs_fp64"] = (extra["gmres_block_jacobi" if pc else "gmres"]["time_to_tol_s"] / tm)
                print(f"bench: {key} refined GMRES {itm} its / {outm} outer {tm:.3f}s relres {rrm:.2e}"
                      + (f", solution error vs FP64 (both to 1e-13) {ent['solution_rel_err_vs_fp64_at_1e-13']:.1e}"
                         if not pc else ""), file=sys.stderr, flush=True)
    extra["mixed"] = mixed
    if not args.no_c2:
        extra["many_rhs"] = bench_c2(B, W, torch, np, stream, args)
    if not args.no_c3:
        extra["batched_uneven"] = bench_c3(B, W, torch, np, args)
    if not args.no_c4:
        extra["learned_precond"] = bench_c4(B, W, torch, np, args)
    if not args.no_maxwell:
        extra["maxwell"] = bench_maxwell(B, W, torch, np, stream, args)
    if args.tune:
        import paper_1906_00785_amd.autotune as AT

        extra["autotune"] = AT.tune(s, q=cfg["q"], eta=cfg["eta"], steps=20)
        print(f"bench: autotune {extra['autotune']['table']}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        cpu = cpu_baseline(cfg, x_host, args.cpu_rows)
        print(f"bench: cpu baseline {cpu['value']:.3e} DOF/s ({time.perf_counter()-t0:.1f}s)", file=sys.stderr,
              flush=True)
        model, ncpu = _cpu_info()
        t0 = time.perf_counter()
        extra["cpu_baseline_openmp"] = cpu_baseline(cfg, x_host, args.cpu_rows, threads=ncpu)
        extra["cpu_baseline_openmp"]["cpu_model"] = model
        print(f"bench: cpu baseline OpenMP ({extra['cpu_baseline_openmp']['cores']} threads) "
              f"{extra['cpu_baseline_openmp']['value']:.3e} DOF/s ({time.perf_counter()-t0:.1f}s)", file=sys.stderr,
              flush=True)
        if not args.no_cpu_legs:
            t0 = time.perf_counter()
            gpu = {"c1_gmres_iterations": extra.get("gmres", {}).get("iterations")}
            extra["cpu_oracle_legs"] = cpu_oracle_legs(args, gpu)
            print(f"bench: oracle legs {time.perf_counter()-t0:.1f}s", file=sys.stderr, flush=True)

    out = {
        "metric": "H2 matvec DOF/s + GMRES time-to-1e-8, mixed/learned vs FP64 plain, 1 GPU",
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "ndof": N, "level": cfg["level"], "degree": cfg["degree"],
                   "q": cfg["q"], "eta": cfg["eta"], "leaf_level": cfg["leaf"], "nfar": info.nfar,
                   "near_nnz": info.near_nnz, "nrhs": 1, "far_field": head},
        "roofline": roof,
        "far_field": head,
        "stages_us": {"near_and_up": stage_ms[0] * 1e3, "coupling": stage_ms[1] * 1e3,
                      "gather_and_down": stage_ms[2] * 1e3, "back": stage_ms[3] * 1e3},
        "other_far_field": {"far_field": "stored_blocks" if head == "on_the_fly" else "on_the_fly",
                            "ms_per_step": ms_st if head == "on_the_fly" else ms_ot,
                            "dof_per_s": N / ((ms_st if head == "on_the_fly" else ms_ot) * 1e-3),
                            "roofline": roof_other,
                            "stages_us": [v * 1e3 for v in (stage_st if head == "on_the_fly" else stage_ot)]},
        "near_gbs": near_bytes / (stage_ms[0] * 1e-3) / 1e9,
        "assembly_s": t_asm,
        "assembly_on_the_fly_s": t_asm_ot,
        "plan_s": t_plan,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
