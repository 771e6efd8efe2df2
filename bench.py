#!/usr/bin/env python
"""Benchmark of the HEX8 finite-element hot path on one MI355X.

Workload: compressible neo-Hookean block, 100x100x100 HEX8 on the unit cube
(1,000,000 elements, 3,090,903 dofs), per-element shear modulus lognormal
(mu = ln 10, sigma = 0.3, seed 0), bulk modulus 10x shear, pulled to stretch 1.2
in 5 load steps, Jacobi-preconditioned Krylov (CG by default: the tangent is SPD;
the paper's BiCGSTAB with --krylov bicgstab) inside Newton.

One timed step = one Newton iteration of load step 5 (starting from the converged
state of load step 4: residual, Dirichlet lifting, tangent assembly, Jacobi
extraction, the Krylov correction solve, the update and the new residual) plus one
adjoint gradient at the converged solution of load step 5 (tangent assembly,
transposed solve with FP64 refinement, per-element VJP) for the objective
J = 1/2 |u_free|^2.  Inputs are resident in HBM before the timed region.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newton-step + adjoint-grad time, 3M-DOF Neo-Hookean; HBM roofline %"
PEAK_HBM_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def spmv_bytes(prob, value_bytes):
    """Algorithmic bytes of one fused Krylov SpMV launch: CSR values, one column index per
    node block (a 16-bit offset from the row node when every neighbour lies within
    +-32767 node numbers, which is when the library stores them so; else 32-bit), node
    row pointers, x gathered once, y written, one dot vector read."""
    nd = prob.spec.ndpn
    n_blocks = prob.nnz // (nd * nd)
    conn = prob.spec.conn
    spread = int((conn.max(axis=1) - conn.min(axis=1)).max()) if conn.size else 0
    idx_bytes = 2 if spread <= 32767 else 4
    return (prob.nnz * value_bytes + n_blocks * idx_bytes + (prob.spec.n_nodes + 1) * 8
            + 3 * prob.n_dofs * value_bytes)


SPMV_PROFILE = os.path.join(ROOT, "profiles", "k_spmv_nodes_nh_tensile_100x100x100.md")
SPMV_SOURCES = ("paper_2212_00964_amd/csrc/linalg.hip", "paper_2212_00964_amd/csrc/internal.h",
                "paper_2212_00964_amd/csrc/lanes.h")


def measured_traffic(nx, ny, nz, precision):
    """HBM bytes per SpMV launch from the committed FETCH_SIZE/WRITE_SIZE summary, or
    None when the summary does not cover this run (other size or precision) or the
    kernel sources changed since the counters were taken."""
    if (nx, ny, nz) != (100, 100, 100) or precision != "mixed" or not os.path.exists(SPMV_PROFILE):
        return None
    fields = {}
    for line in open(SPMV_PROFILE):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.split()[0] if v.split() else ""
    h = hashlib.sha256()
    for f in SPMV_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if fields.get("kernel_source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(gpu_counts, size_z=20, method="cg"):
    """Times the CPU oracle (single-threaded, as written) on a slab of the same workload
    and scales the measured per-unit costs to the full problem and to the iteration
    counts the GPU step performed."""
    from oracle import oracle as orc
    from paper_2212_00964_amd import inputs
    import ctypes
    p = inputs.nh_tensile(100, 100, size_z, L=(1.0, 1.0, size_z / 100.0), n_load_steps=5, seed=0)
    scale = 1_000_000 / p.n_elems
    t0 = time.perf_counter()
    pat = orc.Pattern(p)
    t_pat = time.perf_counter() - t0
    F = orc.load_vector(p)
    u = np.zeros((p.n_nodes, 3))
    u[:, 0] = 0.16 * p.coords[:, 0]  # a stretched state like load step 4
    u = u.ravel()
    t0 = time.perf_counter()
    r = orc.residual(p, pat, u, None, 0.8 * F)
    t_res = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, vals = orc.assemble(p, pat, u, None, None, residual=False)
    t_asm = time.perf_counter() - t0
    its = 10
    x = np.zeros(pat.n)
    it_out, rel = ctypes.c_int(0), ctypes.c_double(0.0)
    b = -r
    t0 = time.perf_counter()
    solver = orc.lib().orc_pcg if method == "cg" else orc.lib().orc_bicgstab
    solver(pat.n, pat.row_ptr, pat.col_idx, vals, b, x, 1e-30, its, ctypes.byref(it_out), ctypes.byref(rel))
    t_it = (time.perf_counter() - t0) / max(it_out.value, 1)
    t0 = time.perf_counter()
    orc.vjp_theta(p, u, x)
    t_vjp = time.perf_counter() - t0
    newton_ms = 1e3 * scale * (2 * t_res + t_asm + gpu_counts["newton_krylov_its"] * t_it)
    adjoint_ms = 1e3 * scale * (t_asm + gpu_counts["adjoint_krylov_its"] * t_it + t_vjp)
    return {"value": newton_ms + adjoint_ms, "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": (f"oracle (plain C, 1 thread) on a {p.shape[0]}x{p.shape[1]}x{p.shape[2]} slab "
                       f"({p.n_elems} elements, {p.n_dofs} dofs) of the same workload: residual {t_res:.2f}s, "
                       f"tangent assembly {t_asm:.2f}s, {method} {1e3 * t_it:.1f} ms/iteration over {it_out.value} "
                       f"iterations, VJP {t_vjp:.2f}s; scaled x{scale:g} to 1M elements and to the GPU step's "
                       f"{gpu_counts['newton_krylov_its']} + {gpu_counts['adjoint_krylov_its']} Krylov iterations "
                       f"(pattern build {t_pat:.1f}s not counted)"),
            "newton_ms": newton_ms, "adjoint_ms": adjoint_ms}


def j2_path(fem, inputs, n: int, nz: int, precond: int = 0) -> dict:
    import torch
    pj = inputs.j2_cylinder(n, nz, n_load_steps=1)
    jp = fem.Problem(pj, "cuda:0")
    # iteration caps far above what the path needs (at most about 4,000 CG iterations per load step
    # with Jacobi, 370 with the two-level preconditioner), so that a failing path ends quickly
    jo = jp.opts(precision=fem.PREC_FP64, krylov=fem.CG, n_load_steps=1, newton_rtol=1e-9, krylov_rtol=1e-6,
                 newton_max_it=50, krylov_max_it=20000 if precond != fem.PRECOND_AMG else 2000, precond=precond)
    pname = "two-level" if precond == fem.PRECOND_AMG else "Jacobi"
    gfull = torch.as_tensor(pj.dirichlet_values, dtype=torch.float64, device="cuda:0")
    uj = torch.zeros(pj.n_dofs, dtype=torch.float64, device="cuda:0")
    n_half = 10
    lam_path = [k / n_half for k in range(1, n_half + 1)] + [1.0 - k / n_half for k in range(1, n_half + 1)]
    szz, newton_j, kry_j = [], [], []
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for lam in lam_path:
            uj, stj = jp.newton_solve(u0=uj, dirichlet_values=lam * gfull, opts=jo)
            szz.append(jp.average_stress()[2])
            newton_j.append(stj.newton_its)
            kry_j.append(stj.krylov_its_total)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        jp.close()
    log(f"J2 path ({pname}): {dt:.2f}s ({1e3 * dt / len(lam_path):.0f} ms/load step), sigma_zz peak {max(szz):.1f} "
        f"end {szz[-1]:.1f}, newton its {sum(newton_j)}, krylov its {sum(kry_j)}")
    return {"workload": f"J2 perfect plasticity, cylinder R 5 H 10 as {n}x{n}x{nz} HEX8 ({pj.n_elems} elements, "
                        f"{pj.n_dofs} dofs), top displacement 0 -> 0.1 -> 0 in 20 load steps, FP64 {pname}-CG "
                        f"(inner rtol 1e-6), Newton rtol 1e-9",
            "s_total": dt, "ms_per_load_step": 1e3 * dt / len(lam_path),
            "top_displacement": [0.1 * x for x in lam_path], "avg_sigma_zz": szz, "newton_its": newton_j,
            "krylov_its": kry_j}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, nargs=3, default=[100, 100, 100])
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--krylov", choices=["cg", "bicgstab"], default="cg")
    ap.add_argument("--precond", choices=["jacobi", "block-jacobi", "two-level"], default="jacobi",
                    help="preconditioner of the timed step (the paper's Jacobi by default)")
    ap.add_argument("--krylov-rtol", type=float, default=1e-3)
    ap.add_argument("--adjoint-rtol", type=float, default=1e-5,
                    help="relative FP64 residual of the adjoint solve; 1e-5 keeps the gradient within ~1e-7 of "
                         "a tight FP64 gradient on this workload (the JSON line reports the measured error)")
    ap.add_argument("--no-compare", action="store_true", help="skip the full FP64-vs-mixed 5-step solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="short run for hardware counters: one bounded Krylov solve (64 iterations) of the "
                         "workload plus a 256 MiB device copy as the counter calibration; prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path is built and measured on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2212_00964_amd import fem, inputs

    torch.cuda.set_device(0)
    nx, ny, nz = args.size
    p = inputs.nh_tensile(nx, ny, nz, n_load_steps=5, seed=0)
    log(f"workload {p.name}: {p.n_elems} elements, {p.n_dofs} dofs on {torch.cuda.get_device_name(0)}")
    t0 = time.perf_counter()
    prob = fem.Problem(p, "cuda:0")
    log(f"pattern + upload {time.perf_counter() - t0:.1f}s, nnz={prob.nnz}")
    prec = fem.PREC_MIXED if args.precision == "mixed" else fem.PREC_FP64
    kry = fem.CG if args.krylov == "cg" else fem.BICGSTAB
    g_final = prob.dirichlet_values

    if args.profile_kernels:
        o = prob.opts(precision=prec, krylov=kry, n_load_steps=1, newton_fixed_its=1, krylov_rtol=1e-12,
                      krylov_max_it=64, check_every=64)
        prob.newton_solve(dirichlet_values=0.2 * g_final, opts=o)
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)  # 256 MiB read + 256 MiB written: calibrates FETCH_SIZE / WRITE_SIZE
        torch.cuda.synchronize()
        log("profile run done")
        prob.close()
        return

    # converged state of load step 4 (schedule 0.2, 0.4, 0.6, 0.8 of the final stretch)
    o4 = prob.opts(precision=prec, krylov=kry, n_load_steps=4, newton_rtol=1e-9, krylov_rtol=args.krylov_rtol)
    t0 = time.perf_counter()
    u4, st4 = prob.newton_solve(dirichlet_values=0.8 * g_final, opts=o4)
    log(f"load steps 1-4: {time.perf_counter() - t0:.2f}s newton_its={st4.newton_its} "
        f"krylov_its={st4.krylov_its_total}")
    o5 = prob.opts(precision=prec, krylov=kry, n_load_steps=1, newton_rtol=1e-9, krylov_rtol=args.krylov_rtol)
    u5, st5 = prob.newton_solve(u0=u4, opts=o5)
    log(f"load step 5: newton_its={st5.newton_its} krylov_its={list(st5.krylov_its[:st5.n_hist])}")
    dJdu = torch.where(prob.mask, torch.zeros_like(u5), u5)

    pc = {"jacobi": fem.PRECOND_JACOBI, "block-jacobi": fem.PRECOND_BLOCK_JACOBI,
          "two-level": fem.PRECOND_AMG}[args.precond]
    step_opts = prob.opts(precision=prec, krylov=kry, n_load_steps=1, newton_fixed_its=1,
                          krylov_rtol=args.krylov_rtol, profile_spmv=1, precond=pc)
    adj_opts = prob.opts(precision=prec, krylov=kry, krylov_rtol=args.krylov_rtol, adjoint_rtol=args.adjoint_rtol,
                         profile_spmv=1, precond=pc)

    def step():
        u, sn = prob.newton_solve(u0=u4, opts=step_opts)
        g, _, sa = prob.adjoint_vjp(u5, dJdu, opts=adj_opts, want_lambda=False)
        return sn, sa, g

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    newton_ms, adj_ms, spmv_ms, spmv_calls, kits_n, kits_a = [], [], 0.0, 0, [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sn, sa, g_step = step()
        newton_ms.append(sn.ms_total)
        adj_ms.append(sa.ms_total)
        spmv_ms += sn.spmv_ms_total + sa.spmv_ms_total
        spmv_calls += sn.spmv_calls + sa.spmv_calls
        kits_n.append(sn.krylov_its_total)
        kits_a.append(sa.krylov_its_total)
    torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    t_newton = float(np.median(newton_ms))
    t_adj = float(np.median(adj_ms))
    log(f"timed: {wall_ms:.2f} ms/step (newton {t_newton:.2f} ms, adjoint {t_adj:.2f} ms), "
        f"krylov its newton={kits_n} adjoint={kits_a}")
    vb = 4 if prec == fem.PREC_MIXED else 8
    avg_spmv_ms = spmv_ms / max(spmv_calls, 1)
    nbytes = spmv_bytes(prob, vb)
    achieved = nbytes / (avg_spmv_ms * 1e-3) / 1e9
    log(f"SpMV: {spmv_calls} timed launches (middle Krylov iteration of every 16), avg {avg_spmv_ms * 1e3:.1f} us, "
        f"{achieved:.0f} GB/s algorithmic")

    out = {
        "metric": METRIC, "value": t_newton + t_adj, "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_ms, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 tangent/SpMV/Krylov + f64 residual/dots" if prec == fem.PREC_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": f"neo-Hookean tensile block {nx}x{ny}x{nz} HEX8 ({p.n_elems} elements, "
                               f"{p.n_dofs} dofs, nnz {prob.nnz}), lognormal G (ln 10, 0.3), kappa = 10 G, "
                               f"load step 5 of 5 to stretch 1.2; {args.precond}-{args.krylov} (inner rtol "
                               f"{args.krylov_rtol:g}), adjoint rtol {args.adjoint_rtol:g}",
                   "precision": args.precision, "parallelism": "single GPU"},
        "newton_step_ms": t_newton, "adjoint_grad_ms": t_adj,
        "dofs_per_s": p.n_dofs / ((t_newton + t_adj) * 1e-3),
        "krylov": args.krylov, "krylov_rtol": args.krylov_rtol, "adjoint_rtol": args.adjoint_rtol,
        "krylov_its": {"newton": int(np.median(kits_n)), "adjoint": int(np.median(kits_a))},
        "roofline": {"bound": "hbm", "kernel": "k_spmv_nodes (fused Krylov SpMV + FP64 dot)", "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": measured_traffic(nx, ny, nz, args.precision),
                     "avg_launch_us": avg_spmv_ms * 1e3, "launches": spmv_calls,
                     "launch_sampling": "HIP events around the SpMV of the middle (9th) Krylov iteration of "
                                        "every 16-iteration check block, over the timed steps",
                     "bytes_per_launch": nbytes},
    }

    if not args.no_compare:
        # FP64 reference gradient (tight), then full 5-step solves of each form
        g_ref, _, _ = prob.adjoint_vjp(u5, dJdu, opts=prob.opts(precision=fem.PREC_FP64, krylov=fem.CG,
                                                                krylov_rtol=1e-8, adjoint_rtol=1e-11),
                                       want_lambda=False)
        out["grad_rel_err_vs_fp64"] = float(torch.linalg.norm(g_step - g_ref) / torch.linalg.norm(g_ref))
        # the same step in the plain FP64 form (same Krylov method and tolerances; its
        # adjoint solve runs to the adjoint tolerance in one sweep, which is the FP64
        # form's fastest setting: restarting at the Newton inner tolerance costs 22% more)
        f_step = prob.opts(precision=fem.PREC_FP64, krylov=kry, n_load_steps=1, newton_fixed_its=1,
                           krylov_rtol=args.krylov_rtol)
        f_adj = prob.opts(precision=fem.PREC_FP64, krylov=kry, krylov_rtol=args.adjoint_rtol,
                          adjoint_rtol=args.adjoint_rtol)
        for _ in range(2):
            _, sf = prob.newton_solve(u0=u4, opts=f_step)
            g_f, _, sfa = prob.adjoint_vjp(u5, dJdu, opts=f_adj, want_lambda=False)
        out["fp64_step"] = {
            "newton_step_ms": sf.ms_total, "adjoint_grad_ms": sfa.ms_total, "value_ms": sf.ms_total + sfa.ms_total,
            "krylov_its": {"newton": sf.krylov_its_total, "adjoint": sfa.krylov_its_total},
            "grad_rel_err_vs_fp64_ref": float(torch.linalg.norm(g_f - g_ref) / torch.linalg.norm(g_ref)),
            "speedup_mixed_over_fp64": (sf.ms_total + sfa.ms_total) / (t_newton + t_adj)}
        log(f"fp64 step: newton {sf.ms_total:.1f} ms, adjoint {sfa.ms_total:.1f} ms, "
            f"speedup of mixed {out['fp64_step']['speedup_mixed_over_fp64']:.2f}x")
        # the same mixed step with the node-block Jacobi preconditioner
        b_step = prob.opts(precision=prec, krylov=kry, n_load_steps=1, newton_fixed_its=1,
                           krylov_rtol=args.krylov_rtol, precond=fem.PRECOND_BLOCK_JACOBI)
        b_adj = prob.opts(precision=prec, krylov=kry, krylov_rtol=args.krylov_rtol, adjoint_rtol=args.adjoint_rtol,
                          precond=fem.PRECOND_BLOCK_JACOBI)
        for _ in range(2):
            _, sb = prob.newton_solve(u0=u4, opts=b_step)
            g_b, _, sba = prob.adjoint_vjp(u5, dJdu, opts=b_adj, want_lambda=False)
        out["block_jacobi_step"] = {
            "newton_step_ms": sb.ms_total, "adjoint_grad_ms": sba.ms_total, "value_ms": sb.ms_total + sba.ms_total,
            "krylov_its": {"newton": sb.krylov_its_total, "adjoint": sba.krylov_its_total},
            "grad_rel_err_vs_fp64_ref": float(torch.linalg.norm(g_b - g_ref) / torch.linalg.norm(g_ref))}
        log(f"block-Jacobi step: newton {sb.ms_total:.1f} ms ({sb.krylov_its_total} its), adjoint {sba.ms_total:.1f} ms "
            f"({sba.krylov_its_total} its)")
        # the same mixed step with the two-level aggregation preconditioner (CG)
        a_step = prob.opts(precision=fem.PREC_MIXED, krylov=fem.CG, n_load_steps=1, newton_fixed_its=1,
                           krylov_rtol=args.krylov_rtol, precond=fem.PRECOND_AMG)
        a_adj = prob.opts(precision=fem.PREC_MIXED, krylov=fem.CG, krylov_rtol=args.krylov_rtol,
                          adjoint_rtol=args.adjoint_rtol, precond=fem.PRECOND_AMG)
        t0 = time.perf_counter()
        n_agg, n_cb = prob.amg_sizes()
        t_setup = time.perf_counter() - t0
        for _ in range(2):
            _, sm = prob.newton_solve(u0=u4, opts=a_step)
            g_m, _, sma = prob.adjoint_vjp(u5, dJdu, opts=a_adj, want_lambda=False)
        out["two_level_step"] = {
            "newton_step_ms": sm.ms_total, "adjoint_grad_ms": sma.ms_total, "value_ms": sm.ms_total + sma.ms_total,
            "krylov_its": {"newton": sm.krylov_its_total, "adjoint": sma.krylov_its_total},
            "refresh_ms_per_tangent": sm.ms_assemble,
            "grad_rel_err_vs_fp64_ref": float(torch.linalg.norm(g_m - g_ref) / torch.linalg.norm(g_ref)),
            "aggregates": n_agg, "coarse_blocks": n_cb, "setup_s": t_setup,
            "speedup_over_jacobi": (t_newton + t_adj) / (sm.ms_total + sma.ms_total)}
        log(f"two-level step: newton {sm.ms_total:.1f} ms ({sm.krylov_its_total} its), adjoint {sma.ms_total:.1f} ms "
            f"({sma.krylov_its_total} its); {out['two_level_step']['speedup_over_jacobi']:.2f}x the Jacobi step")
        u_ref, _ = prob.newton_solve(opts=prob.opts(precision=fem.PREC_FP64, krylov=fem.CG, krylov_rtol=1e-8,
                                                    newton_rtol=1e-11))
        res = {}
        forms = (("mixed-" + args.krylov, prec if prec == fem.PREC_MIXED else fem.PREC_MIXED, kry, args.krylov_rtol,
                  fem.PRECOND_JACOBI),
                 ("fp64-cg", fem.PREC_FP64, fem.CG, args.krylov_rtol, fem.PRECOND_JACOBI),
                 ("fp64-bicgstab", fem.PREC_FP64, fem.BICGSTAB, args.krylov_rtol, fem.PRECOND_JACOBI),
                 ("mixed-cg-two-level", fem.PREC_MIXED, fem.CG, args.krylov_rtol, fem.PRECOND_AMG))
        for name, pr, kr, eta, pc in forms:
            o = prob.opts(precision=pr, krylov=kr, newton_rtol=1e-9, krylov_rtol=eta, precond=pc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, st = prob.newton_solve(opts=o)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            err = float(torch.linalg.norm(u - u_ref) / torch.linalg.norm(u_ref))
            res[name] = {"s": dt, "newton_its": st.newton_its, "krylov_its": st.krylov_its_total,
                         "rel_err_vs_tight_fp64": err}
            log(f"full 5-step solve {name}: {dt:.2f}s newton_its={st.newton_its} krylov_its={st.krylov_its_total} "
                f"err={err:.2e}")
        # SIMP compliance optimisation iterations on the 120x60x30 cantilever (216,000
        # elements): solve + compliance + adjoint VJP + sensitivity filter + MMA step
        from paper_2212_00964_amd.topopt import SimpCompliance
        ps = inputs.simp_cantilever(120, 60, 30)
        for key, pcs in (("simp_loop", fem.PRECOND_JACOBI), ("simp_loop_two_level", fem.PRECOND_AMG)):
            sp = fem.Problem(ps, "cuda:0")
            so = sp.opts(precision=fem.PREC_MIXED, krylov=fem.CG, n_load_steps=1, newton_rtol=1e-9, krylov_rtol=1e-3,
                         precond=pcs)
            opt = SimpCompliance(sp, rmin=1.5 * (2.0 / 120), vfrac=0.5, solve_opts=so)
            opt.step()  # warm-up iteration (its compliance is kept in the history)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n_opt = 4
            opt.run(n_opt)
            torch.cuda.synchronize()
            ms_it = 1e3 * (time.perf_counter() - t0) / n_opt
            pname = "Jacobi" if pcs == fem.PRECOND_JACOBI else "two-level"
            out[key] = {"workload": "SIMP cantilever 120x60x30 HEX8 on 2x1x0.5 (216000 elements, 686433 dofs), "
                                    f"theta0 ~ U(0.4, 0.6), rmin 1.5 h, material fraction 0.5, mixed-precision {pname} CG",
                        "ms_per_iteration": ms_it, "compliance": opt.compliance, "material_fraction": opt.volume,
                        "krylov_its": [s_.krylov_its_total for s_ in opt.stats]}
            log(f"SIMP loop ({pname}): {ms_it:.1f} ms/iteration, compliance {[round(c, 4) for c in opt.compliance]}")
            sp.close()
        # full-field inference: L-BFGS over the nodal source of a Poisson problem on the
        # 1 x 1 x 0.2 box, 50x50x10 HEX8, 250 observed nodes (observations synthesised by
        # the forward solve at the true bimodal source)
        from paper_2212_00964_amd.inference import SourceInference, lbfgs
        pi, obs_idx = inputs.poisson_inference(50, 50, 10, n_obs=250, seed=1)
        ip = fem.Problem(pi, "cuda:0")
        b_true = torch.as_tensor(pi.source_nodal, dtype=torch.float64, device="cuda:0")
        setup = SourceInference(ip, obs_idx, torch.zeros(len(obs_idx), dtype=torch.float64))
        u_true = setup.solve(b_true).clone()
        fun = SourceInference(ip, obs_idx, u_true[torch.as_tensor(obs_idx, device="cuda:0")].clone())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_lb = 20
        hx, hJ = lbfgs(fun, torch.zeros(pi.n_nodes, dtype=torch.float64, device="cuda:0"), n_lb)
        torch.cuda.synchronize()
        ms_lb = 1e3 * (time.perf_counter() - t0) / n_lb
        u_pred = fun.solve(hx[-1])
        field_err = float(torch.linalg.norm(u_pred - u_true) / torch.linalg.norm(u_true))
        out["inference_loop"] = {"workload": "Poisson source inference 50x50x10 HEX8 on 1x1x0.2 (26,901 dofs), "
                                             "250 observed nodes, L-BFGS from theta = 0, FP64 CG solves",
                                 "ms_per_iteration": ms_lb, "objective": hJ, "forward_and_adjoint_solves": fun.n_solves,
                                 "field_rel_err": field_err}
        log(f"inference: {ms_lb:.1f} ms/iteration, J {hJ[0]:.3e} -> {hJ[-1]:.3e}, field error {field_err:.3f}")
        ip.close()
        # perfect J2 plasticity: the cylinder of radius 5 and height 10 (bottom fixed, top
        # moved along z) loaded to 0.1 in 10 load steps and unloaded to 0 in 10 more,
        # E = 70e3, nu = 0.3, sigma_y = 250; one fem_newton_solve call per load step so
        # that the averaged stress is recorded after each.  FP64 path: past the limit load
        # the consistent tangent's smallest stiffness falls below FP32 rounding of its
        # deviatoric projection and FP32 CG meets an indefinite matrix.
        for key, pcj in (("plasticity_path", fem.PRECOND_JACOBI), ("plasticity_path_two_level", fem.PRECOND_AMG)):
            try:
                out[key] = j2_path(fem, inputs, 48, 96, pcj)
            except fem.FemError as e:
                out[key] = {"error": str(e)}
                log(f"J2 path failed: {e}")
        mixed_name = forms[0][0]
        res["speedup_mixed_over_fp64_cg"] = res["fp64-cg"]["s"] / res[mixed_name]["s"]
        res["speedup_mixed_over_fp64_bicgstab"] = res["fp64-bicgstab"]["s"] / res[mixed_name]["s"]
        out["full_solve"] = res

    prob.close()
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline({"newton_krylov_its": int(np.median(kits_n)),
                                            "adjoint_krylov_its": int(np.median(kits_a))}, method=args.krylov)
        log(f"cpu baseline {time.perf_counter() - t0:.1f}s: {out['cpu_baseline']['value']:.0f} ms")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
