#!/usr/bin/env python
"""Benchmark of the HEX8 finite-element hot path on one MI355X.

Workload: compressible neo-Hookean block, 100x100x100 HEX8 on the unit cube
(1,000,000 elements, 3,090,903 dofs), per-element shear modulus lognormal
(mu = ln 10, sigma = 0.3, seed 0), bulk modulus 10x shear, pulled to stretch 1.2
in 5 load steps, Newton with Jacobi-preconditioned BiCGSTAB in mixed precision (the
workload's named form: the tangent assembled and stored in FP32, the Krylov vectors in
FP64, FP64 residuals and refinement; --precision mixed keeps the Krylov vectors in
FP32, --precision fp64 is the plain FP64 form, --krylov cg for Jacobi-CG).

One timed step solves load step 5 from the converged state of load step 4 (every
Newton iteration timed: FP64 residual, Dirichlet lifting, tangent assembly, Jacobi
extraction, the Krylov correction solve, the update and the new residual) and takes
the adjoint gradient at its solution (tangent assembly, transposed solve with FP64
refinement, per-element VJP) for J = 1/2 |u_free|^2.  The reported value is
T_step + T_grad with T_step the median Newton iteration.  Inputs are resident in HBM
before the timed region.

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


def spmv_bytes(prob, value_bytes, vector_bytes=None):
    """Algorithmic bytes of one Krylov SpMV launch (the node-block form): the values,
    one 32-bit column index per node block, the node row pointers, x gathered once,
    y written and one dot-product vector read."""
    nd = prob.spec.ndpn
    n_blocks = prob.nnz // (nd * nd)
    vb = value_bytes if vector_bytes is None else vector_bytes
    return prob.nnz * value_bytes + n_blocks * 4 + (prob.spec.n_nodes + 1) * 8 + 3 * prob.n_dofs * vb


def assembly_bytes(prob, value_bytes):
    """Minimum bytes of a tangent assembly: every value written once, u, theta,
    coordinates and connectivity read once."""
    sp = prob.spec
    return prob.nnz * value_bytes + prob.n_dofs * 8 + sp.n_elems * 8 + sp.n_nodes * 24 + sp.n_elems * 32


PROFILE_DIR = os.path.join(ROOT, "profiles")
KRYLOV_SOURCES = ("paper_2212_00964_amd/csrc/linalg.hip", "paper_2212_00964_amd/csrc/internal.h",
                  "paper_2212_00964_amd/csrc/lanes.h")
ASSEMBLY_SOURCES = ("paper_2212_00964_amd/csrc/element.hip", "paper_2212_00964_amd/csrc/internal.h",
                    "paper_2212_00964_amd/csrc/lanes.h")


def sources_sha(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(profile, sources):
    """HBM bytes per launch from a committed FETCH_SIZE/WRITE_SIZE summary, or None when
    the summary is missing or the kernel sources changed since the counters were taken."""
    path = os.path.join(PROFILE_DIR, profile)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.split()[0] if v.split() else ""
    if fields.get("kernel_source_sha256") != sources_sha(sources) or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(gpu_counts, method):
    """The CPU oracle (plain C, OpenMP loops on all host threads) timed on the full
    workload: the FP64 residual, the tangent assembly, one Krylov iteration and the
    per-element VJP, each the median of 3 runs, combined with the iteration counts of
    the GPU's plain FP64 form of the same step (the same FP64 algorithm)."""
    from oracle import oracle as orc
    from paper_2212_00964_amd import inputs
    import ctypes
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    model, ncpu = host_cpu()
    p = inputs.nh_tensile(100, 100, 100, n_load_steps=5, seed=0)
    med = lambda xs: float(np.median(xs))  # noqa: E731
    with orc.threads(threads):
        t0 = time.perf_counter()
        pat = orc.Pattern(p)
        t_pat = time.perf_counter() - t0
        F = orc.load_vector(p)
        u = np.zeros((p.n_nodes, 3))
        u[:, 0] = 0.16 * p.coords[:, 0]  # a stretched state like load step 4
        u = u.ravel()
        t_res, t_asm, t_it, t_vjp, t_spmv = [], [], [], [], []
        its_per_run = 5
        solver = orc.lib().orc_pcg if method == "cg" else orc.lib().orc_bicgstab
        for _ in range(3):
            t0 = time.perf_counter()
            r = orc.residual(p, pat, u, None, 0.8 * F)
            t_res.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            _, vals = orc.assemble(p, pat, u, None, None, residual=False)
            t_asm.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            orc.spmv(pat, vals, r)
            t_spmv.append(time.perf_counter() - t0)
            x = np.zeros(pat.n)
            it_out, rel = ctypes.c_int(0), ctypes.c_double(0.0)
            t0 = time.perf_counter()
            solver(pat.n, pat.row_ptr, pat.col_idx, vals, -r, x, 1e-30, its_per_run, ctypes.byref(it_out),
                   ctypes.byref(rel))
            t_it.append((time.perf_counter() - t0) / max(it_out.value, 1))
            t0 = time.perf_counter()
            orc.vjp_theta(p, u, x)
            t_vjp.append(time.perf_counter() - t0)
            del vals
    tr, ta, ti, tv, tm = med(t_res), med(t_asm), med(t_it), med(t_vjp), med(t_spmv)
    small = small_cpu_timings()
    # Newton iteration: residual, tangent, the Krylov solve, the residual after the update;
    # gradient: tangent, the Krylov solve, one refinement residual per sweep, the VJP
    newton_ms = 1e3 * (2 * tr + ta + gpu_counts["newton_krylov_its"] * ti)
    adjoint_ms = 1e3 * (ta + gpu_counts["adjoint_krylov_its"] * ti + gpu_counts["adjoint_sweeps"] * tr + tv)
    return {"value": newton_ms + adjoint_ms, "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": (f"oracle (plain C FP64, OpenMP on {threads} threads of a {ncpu}-CPU host, {model}) on the full "
                       f"100x100x100 workload: residual {tr:.2f} s, tangent assembly {ta:.2f} s, {method} "
                       f"{1e3 * ti:.1f} ms per iteration ({its_per_run} iterations per run), VJP {tv:.2f} s, each the "
                       f"median of 3 runs; combined with the iteration counts of the GPU's plain FP64 form of the "
                       f"same step ({gpu_counts['newton_krylov_its']} Krylov iterations for the median Newton "
                       f"iteration, {gpu_counts['adjoint_krylov_its']} in {gpu_counts['adjoint_sweeps']} adjoint "
                       f"sweeps); pattern build {t_pat:.1f} s not counted"),
            "newton_ms": newton_ms, "adjoint_ms": adjoint_ms,
            "residual_s": tr, "assembly_s": ta, "spmv_ms": 1e3 * tm, "krylov_iteration_ms": 1e3 * ti, "vjp_s": tv,
            "host": {"model": model, "logical_cpus": ncpu, "sockets": host_sockets(), "threads_used": threads},
            "single_thread_small_workloads": small}


def host_sockets():
    ids = set()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("physical id"):
                ids.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    return len(ids) or None


def small_cpu_timings():
    """The oracle on one thread for the two small workloads (8^3 Poisson, 64x32x32
    cantilever): tangent assembly, one SpMV and, for the Poisson cube, the whole Jacobi-CG
    solve; medians of 3 runs."""
    from oracle import oracle as orc
    from paper_2212_00964_amd import inputs
    med = lambda xs: float(np.median(xs))  # noqa: E731
    out = {}
    with orc.threads(1):
        for name, p in (("poisson_8x8x8", inputs.workload(1)), ("cantilever_64x32x32", inputs.workload(2))):
            pat = orc.Pattern(p)
            F = orc.load_vector(p)
            u = np.zeros(p.n_dofs)
            ta, tm, ts = [], [], []
            for _ in range(3):
                t0 = time.perf_counter()
                r, vals = orc.assemble(p, pat, u, None, F)
                ta.append(time.perf_counter() - t0)
                t0 = time.perf_counter()
                orc.spmv(pat, vals, r)
                tm.append(time.perf_counter() - t0)
                if name.startswith("poisson"):
                    t0 = time.perf_counter()
                    _, cg_its, _ = orc.krylov(pat, vals, -r, "cg", rtol=1e-10)
                    ts.append(time.perf_counter() - t0)
            out[name] = {"dofs": int(p.n_dofs), "nnz": int(pat.col_idx.size), "assembly_ms": 1e3 * med(ta),
                         "spmv_ms": 1e3 * med(tm)}
            if ts:  # the manufactured sine load is an eigenvector of the Jacobi-scaled operator here
                out[name].update({"cg_solve_ms": 1e3 * med(ts), "cg_iterations": cg_its})
    return out


def refine_for(fem, prec, kry):
    """FP64-refined corrections for mixed BiCGSTAB: FP32 sweeps that each halve the FP64
    residual and restart from it (FP32 BiCGSTAB asked for three decades at once stalls on
    the smooth right-hand sides of late Newton iterations; sweeps of 0.2, 0.3 and 0.5 all
    bring the 5-step solve from 17,137 to about 7,000 iterations, 0.5 also helps the
    adjoint).  CG keeps one solve per correction (restarts would discard its Krylov space)."""
    return 0.5 if (prec == fem.PREC_MIXED and kry == fem.BICGSTAB) else 0.0


def adjoint_rtol_for(fem, kry, given):
    """Adjoint tolerance: both Krylov methods reach a gradient within 1e-6 of a tight FP64
    gradient, CG at 1e-5 (it minimises the error in the energy norm) and BiCGSTAB only at
    1e-6 (2e-6 to 5e-6 at 1e-5, measured on this workload)."""
    if given is not None:
        return given
    return 1e-5 if kry == fem.CG else 1e-6


def measure_form(fem, prob, u4, prec, kry, pc, krylov_rtol, adjoint_rtol, steps, warmup, profile=False,
                 u_obs=None, krylov_max_it=20000, newton_max_it=50):
    """Load step 5 solved from the converged state of load step 4 (every Newton
    iteration timed) and the adjoint gradient at its solution of J = 1/2 |u_free|^2, or of
    the misfit J = 1/2 |u_free - u_obs|^2 when u_obs is given.
    T_step = median Newton iteration, T_grad = the gradient."""
    import torch
    rr = refine_for(fem, prec, kry)
    adjoint_rtol = adjoint_rtol_for(fem, kry, adjoint_rtol)
    step_o = prob.opts(precision=prec, krylov=kry, n_load_steps=1, newton_rtol=1e-9, newton_max_it=newton_max_it,
                       krylov_rtol=krylov_rtol, profile_spmv=int(profile), precond=pc, refine_rtol=rr,
                       krylov_max_it=krylov_max_it)
    # sweeps that each halve the residual need about 20 for 1e-6: leave room
    adj_o = prob.opts(precision=prec, krylov=kry, krylov_rtol=krylov_rtol, adjoint_rtol=adjoint_rtol,
                      profile_spmv=int(profile), precond=pc, refine_rtol=rr, adjoint_max_refine=60,
                      krylov_max_it=krylov_max_it)

    def one():
        u5, sn = prob.newton_solve(u0=u4, opts=step_o)
        dJdu = torch.where(prob.mask, torch.zeros_like(u5), u5 if u_obs is None else u5 - u_obs)
        g, _, sa = prob.adjoint_vjp(u5, dJdu, opts=adj_o, want_lambda=False)
        return u5, sn, sa, g

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [one() for _ in range(steps)]
    torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t0) / max(steps, 1)
    it_ms = [list(r[1].iter_ms[:r[1].n_hist]) for r in recs]
    its = [list(r[1].krylov_its[:r[1].n_hist]) for r in recs]
    t_step = float(np.median([np.median(x) for x in it_ms]))
    t_grad = float(np.median([r[2].ms_total for r in recs]))
    last = recs[-1]
    return {"t_step": t_step, "t_grad": t_grad, "wall_ms": wall_ms, "iter_ms": it_ms[-1], "krylov_its": its[-1],
            "median_iteration_krylov_its": int(np.median(its[-1])),
            "adjoint_krylov_its": last[2].krylov_its_total, "adjoint_sweeps": last[2].newton_its,
            "spmv_ms": sum(r[1].spmv_ms_total + r[2].spmv_ms_total for r in recs),
            "spmv_calls": sum(r[1].spmv_calls + r[2].spmv_calls for r in recs),
            "u5": last[0], "g": last[3]}


def assembly_roofline(fem, prob, u, reps=5):
    """FP32 tangent assembly (element tangents + node gather), HIP events on the stream
    the library uses (torch's current stream)."""
    import torch
    vals = torch.empty(prob.nnz, dtype=torch.float32, device="cuda:0")
    ws = prob.workspace(None)
    L = fem.lib()
    args = (prob.handle, fem._ptr(u), fem._ptr(prob.theta), None, fem._ptr(vals), fem.F32, fem.LAYOUT_CSR,
            fem._ptr(ws), ws.numel(), fem._stream())
    fem._check(L.fem_assemble(*args))
    prob.check()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fem._check(L.fem_assemble(*args))
        b.record()
    prob.check()
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    nbytes = assembly_bytes(prob, 4)
    achieved = nbytes / (ms * 1e-3) / 1e9
    del vals
    return {"bound": "hbm", "kernel": "k_element_tangent + k_gather_node (FP32 values, CSR)", "achieved": achieved,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "traffic": measured_traffic("assembly_nh_tensile_100x100x100.md", ASSEMBLY_SOURCES),
            "avg_launch_us": 1e3 * ms, "launches": reps, "bytes_per_launch": nbytes,
            "note": "minimum bytes (values once; u, theta, coordinates, connectivity once); the two-pass design "
                    "also writes and reads back the element blocks"}


def j2_path(fem, inputs, n: int, nz: int, precond: int = 0, precision: int = 0, max_bisections: int = 0,
            time_limit_s: float = 0.0) -> dict:
    import torch
    pj = inputs.j2_cylinder(n, nz, n_load_steps=1)
    jp = fem.Problem(pj, "cuda:0")
    # iteration caps far above what the path needs (at most about 4,000 CG iterations per load step
    # with Jacobi, 370 with the two-level preconditioner), so that a failing path ends quickly; with
    # the recovery on, a failed attempt must end fast, so the caps are tighter
    recover = max_bisections > 0
    jo = jp.opts(precision=precision, krylov=fem.CG, n_load_steps=1, newton_rtol=1e-9, krylov_rtol=1e-6,
                 newton_max_it=15 if recover else 50,
                 krylov_max_it=(6000 if recover else 20000) if precond != fem.PRECOND_AMG else 2000, precond=precond,
                 max_bisections=max_bisections)
    pname = "two-level" if precond == fem.PRECOND_AMG else "Jacobi"
    gfull = torch.as_tensor(pj.dirichlet_values, dtype=torch.float64, device="cuda:0")
    uj = torch.zeros(pj.n_dofs, dtype=torch.float64, device="cuda:0")
    n_half = 10
    lam_path = [k / n_half for k in range(1, n_half + 1)] + [1.0 - k / n_half for k in range(1, n_half + 1)]
    szz, newton_j, kry_j, bis_j = [], [], [], []
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for step, lam in enumerate(lam_path):
            if time_limit_s and time.perf_counter() - t0 > time_limit_s:
                raise TimeoutError(f"stopped after {step} of {len(lam_path)} load steps ({time_limit_s:g} s budget)")
            uj, stj = jp.newton_solve(u0=uj, dirichlet_values=lam * gfull, opts=jo)
            if recover:
                log(f"J2 path with recovery: load step {step + 1}: newton {stj.newton_its}, krylov {stj.krylov_its_total}, "
                    f"halvings {stj.bisections}")
            szz.append(jp.average_stress()[2])
            newton_j.append(stj.newton_its)
            kry_j.append(stj.krylov_its_total)
            bis_j.append(stj.bisections)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        jp.close()
    log(f"J2 path ({pname}): {dt:.2f}s ({1e3 * dt / len(lam_path):.0f} ms/load step), sigma_zz peak {max(szz):.1f} "
        f"end {szz[-1]:.1f}, newton its {sum(newton_j)}, krylov its {sum(kry_j)}")
    return {"workload": f"J2 perfect plasticity, cylinder R 5 H 10 as {n}x{n}x{nz} HEX8 ({pj.n_elems} elements, "
                        f"{pj.n_dofs} dofs), top displacement 0 -> 0.1 -> 0 in 20 load steps, "
                        f"{'mixed' if precision else 'FP64'} {pname}-CG (inner rtol 1e-6), Newton rtol 1e-9"
                        + (f", load-step recovery up to {max_bisections} halvings" if max_bisections else ""),
            "s_total": dt, "ms_per_load_step": 1e3 * dt / len(lam_path),
            "top_displacement": [0.1 * x for x in lam_path], "avg_sigma_zz": szz, "newton_its": newton_j,
            "krylov_its": kry_j, "bisections": bis_j}


def next_rows(fem, inputs, out):
    """The NEXT rows measured beside the benchmark line: the SIMP loop, full-field
    inference and the J2 loading-unloading path."""
    import torch
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
    # FP64 (the benchmark's J2 form), and the mixed form with the load-step recovery on:
    # past the limit load the FP32 tangent can be indefinite, which CG reports as
    # FEM_EBREAKDOWN; the recovery halves the step up to 4 times, and the row records
    # either the converged path or the error it ends with
    for key, pcj, prj, nb in (("plasticity_path", fem.PRECOND_JACOBI, fem.PREC_FP64, 0),
                              ("plasticity_path_two_level", fem.PRECOND_AMG, fem.PREC_FP64, 0),
                              ("plasticity_path_mixed_recovery", fem.PRECOND_JACOBI, fem.PREC_MIXED, 3)):
        try:
            out[key] = j2_path(fem, inputs, 48, 96, pcj, prj, nb, time_limit_s=40.0 if nb else 0.0)
        except (fem.FemError, TimeoutError) as e:
            out[key] = {"error": str(e), "code": getattr(e, "name", "time budget"),
                        "form": f"{'mixed' if prj else 'FP64'} Jacobi-CG, max_bisections {nb}"}
            log(f"J2 path ({key}) ended with {e}")


def linear_workload(fem, inputs, which, steps, warmup):
    """The linear workloads (64x32x32 cantilever, FP64 vs mixed; 120x60x30 SIMP cantilever):
    the full solve to a 1e-9 relative residual and the adjoint gradient (J = 1/2 |u_free|^2,
    or the compliance F.u for SIMP) in every form, each timed over `steps` repetitions."""
    import torch
    p = inputs.workload(2 if which == "cantilever" else 4)
    prob = fem.Problem(p, "cuda:0")
    log(f"workload {p.name}: {p.n_elems} elements, {p.n_dofs} dofs, nnz {prob.nnz}")
    F = prob.load_vector()
    ref_o = prob.opts(precision=fem.PREC_FP64, krylov=fem.CG, n_load_steps=1, newton_rtol=1e-11, krylov_rtol=1e-10,
                      adjoint_rtol=1e-11, adjoint_max_refine=20)
    u_ref, _ = prob.newton_solve(opts=ref_o)

    def dJdu_of(u):
        return F.clone() if which == "simp" else torch.where(prob.mask, torch.zeros_like(u), u)

    g_ref, _, _ = prob.adjoint_vjp(u_ref, dJdu_of(u_ref), opts=ref_o, want_lambda=False)
    rows = {}
    for name, prec, kry in (("fp64-cg", fem.PREC_FP64, fem.CG), ("mixed-cg", fem.PREC_MIXED, fem.CG),
                            ("mixed64-cg", fem.PREC_MIXED_V64, fem.CG),
                            ("fp64-bicgstab", fem.PREC_FP64, fem.BICGSTAB),
                            ("mixed-bicgstab", fem.PREC_MIXED, fem.BICGSTAB),
                            ("mixed64-bicgstab", fem.PREC_MIXED_V64, fem.BICGSTAB)):
        rr = refine_for(fem, prec, kry)
        so = prob.opts(precision=prec, krylov=kry, n_load_steps=1, newton_rtol=1e-9, krylov_rtol=1e-3, refine_rtol=rr,
                       krylov_max_it=20000)
        ao = prob.opts(precision=prec, krylov=kry, krylov_rtol=1e-3, adjoint_rtol=adjoint_rtol_for(fem, kry, None),
                       refine_rtol=rr, adjoint_max_refine=60, krylov_max_it=20000)
        solve_ms, grad_ms = [], []
        try:
            for k in range(warmup + steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                u, st = prob.newton_solve(opts=so)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                g, _, sa = prob.adjoint_vjp(u, dJdu_of(u), opts=ao, want_lambda=False)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                if k >= warmup:
                    solve_ms.append(1e3 * (t1 - t0))
                    grad_ms.append(1e3 * (t2 - t1))
        except fem.FemError as e:  # recorded: the other forms still run
            rows[name] = {"error": str(e)}
            log(f"{name}: {e}")
            continue
        rows[name] = {"solve_ms": float(np.median(solve_ms)), "grad_ms": float(np.median(grad_ms)),
                      "newton_its": st.newton_its, "krylov_its": st.krylov_its_total,
                      "adjoint_krylov_its": sa.krylov_its_total,
                      "u_rel_err": float(torch.linalg.norm(u - u_ref) / torch.linalg.norm(u_ref)),
                      "grad_rel_err": float(torch.linalg.norm(g - g_ref) / torch.linalg.norm(g_ref))}
        log(f"{name}: solve {rows[name]['solve_ms']:.1f} ms ({st.krylov_its_total} its), gradient "
            f"{rows[name]['grad_ms']:.1f} ms ({sa.krylov_its_total} its), errors {rows[name]['u_rel_err']:.1e} / "
            f"{rows[name]['grad_rel_err']:.1e}")
    prob.close()
    print(json.dumps({"workload": f"{p.name} ({p.n_elems} elements, {p.n_dofs} dofs, nnz {prob.nnz}); solve to a 1e-9 "
                                  f"relative residual and the adjoint gradient of "
                                  + ("the compliance F.u" if which == "simp" else "J = 1/2 |u_free|^2"),
                      "steps": steps, "warmup": warmup, "forms": rows}), flush=True)


def summarize_trace(path, out_path):
    """Per-kernel dispatch statistics from a rocprofv3 kernel trace (CSV): count, median,
    mean and total duration.  The median is what the profile summaries quote: Krylov
    launches that find the solve already converged exit at once and pull the mean down."""
    import csv
    import collections
    per = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            per[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    with open(out_path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "MedianUs", "MeanUs", "MinUs", "MaxUs", "TotalUs"])
        for name, ds in sorted(per.items(), key=lambda kv: -sum(kv[1])):
            ds = sorted(ds)
            w.writerow([name, len(ds), ds[len(ds) // 2], sum(ds) / len(ds), ds[0], ds[-1], sum(ds)])


def main():
    if len(sys.argv) == 4 and sys.argv[1] == "--summarize-trace":
        summarize_trace(sys.argv[2], sys.argv[3])
        return
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["nh100", "inverse", "cantilever", "simp"], default="nh100",
                    help="nh100: the 100^3 neo-Hookean block (the benchmark line); inverse: the 200x100x100 "
                         "inverse-modulus block (misfit objective); cantilever / simp: the linear 64x32x32 and "
                         "120x60x30 workloads, every form (a JSON line of their own)")
    ap.add_argument("--size", type=int, nargs=3, default=None)
    ap.add_argument("--precision", choices=["mixed", "mixed64", "fp64"], default="mixed64",
                    help="mixed: FP32 tangent and FP32 Krylov vectors; mixed64: FP32 tangent under FP64 Krylov "
                         "vectors; fp64")
    ap.add_argument("--krylov", choices=["cg", "bicgstab"], default="bicgstab",
                    help="Krylov method of the timed step (the workload names Jacobi-BiCGSTAB)")
    ap.add_argument("--precond", choices=["jacobi", "block-jacobi", "two-level"], default="jacobi",
                    help="preconditioner of the timed step (the paper's Jacobi by default)")
    ap.add_argument("--krylov-rtol", type=float, default=1e-3)
    ap.add_argument("--adjoint-rtol", type=float, default=None,
                    help="relative FP64 residual of the adjoint solve (default 1e-6 for BiCGSTAB, 1e-5 for CG: "
                         "each keeps the gradient within 1e-6 of a tight FP64 gradient on this workload; the "
                         "JSON line reports the measured error)")
    ap.add_argument("--no-compare", action="store_true", help="skip the other forms, full solves and NEXT rows")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="short run for hardware counters: one bounded Krylov solve (64 iterations) of the "
                         "workload, one tangent assembly, plus a 256 MiB device copy as the counter calibration; "
                         "prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path is built and measured on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2212_00964_amd import fem, inputs

    torch.cuda.set_device(0)
    if args.workload in ("cantilever", "simp"):
        linear_workload(fem, inputs, args.workload, args.steps, args.warmup)
        return
    if args.workload == "inverse":
        nx, ny, nz = args.size or (200, 100, 100)
        p, theta_true = inputs.nh_inverse(nx, ny, nz)
    else:
        nx, ny, nz = args.size or (100, 100, 100)
        p, theta_true = inputs.nh_tensile(nx, ny, nz, n_load_steps=5, seed=0), None
    log(f"workload {p.name}: {p.n_elems} elements, {p.n_dofs} dofs on {torch.cuda.get_device_name(0)}")
    t0 = time.perf_counter()
    prob = fem.Problem(p, "cuda:0")
    log(f"pattern + upload {time.perf_counter() - t0:.1f}s, nnz={prob.nnz}")
    prec = {"mixed": fem.PREC_MIXED, "mixed64": fem.PREC_MIXED_V64, "fp64": fem.PREC_FP64}[args.precision]
    if args.precond == "two-level" and prec == fem.PREC_MIXED_V64:
        raise SystemExit("the two-level preconditioner runs with --precision mixed or fp64")
    kry = fem.CG if args.krylov == "cg" else fem.BICGSTAB
    pc = {"jacobi": fem.PRECOND_JACOBI, "block-jacobi": fem.PRECOND_BLOCK_JACOBI,
          "two-level": fem.PRECOND_AMG}[args.precond]
    g_final = prob.dirichlet_values

    if args.profile_kernels:
        o = prob.opts(precision=prec, krylov=kry, n_load_steps=1, newton_fixed_its=1, krylov_rtol=1e-12,
                      krylov_max_it=64, check_every=64, precond=pc)
        u, _ = prob.newton_solve(dirichlet_values=0.2 * g_final, opts=o)
        prob.assemble(u, residual=False, values_dtype=torch.float64 if prec == fem.PREC_FP64 else torch.float32)
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)  # 256 MiB read + 256 MiB written: calibrates FETCH_SIZE / WRITE_SIZE
        torch.cuda.synchronize()
        log("profile run done")
        prob.close()
        return

    # converged state of load step 4 (schedule 0.2, 0.4, 0.6, 0.8 of the final stretch), in
    # the timed form; the inverse workload's objective is the misfit to the forward solution
    # at theta_true, its gradient taken at the uniform theta
    o4 = prob.opts(precision=prec, krylov=kry, n_load_steps=4, newton_rtol=1e-9, krylov_rtol=args.krylov_rtol,
                   precond=pc, refine_rtol=refine_for(fem, prec, kry))
    u_obs = None
    if theta_true is not None:
        u_obs, _ = prob.newton_solve(theta=theta_true, opts=prob.opts(precision=prec, krylov=kry, newton_rtol=1e-9,
                                                                       krylov_rtol=args.krylov_rtol, precond=pc,
                                                                       refine_rtol=refine_for(fem, prec, kry)))
    t0 = time.perf_counter()
    u4, st4 = prob.newton_solve(dirichlet_values=0.8 * g_final, opts=o4)
    log(f"load steps 1-4: {time.perf_counter() - t0:.2f}s newton_its={st4.newton_its} "
        f"krylov_its={st4.krylov_its_total}")

    def objective_grad(u5):
        return torch.where(prob.mask, torch.zeros_like(u5), u5 if u_obs is None else u5 - u_obs)

    def measure(pr, kr, pcn, steps, warmup, profile=False, krylov_max_it=20000, newton_max_it=50):
        return measure_form(fem, prob, u4, pr, kr, pcn, args.krylov_rtol, args.adjoint_rtol, steps, warmup, profile,
                            u_obs=u_obs, krylov_max_it=krylov_max_it, newton_max_it=newton_max_it)

    main_form = measure(prec, kry, pc, args.steps, args.warmup, profile=True)
    t_step, t_grad = main_form["t_step"], main_form["t_grad"]
    log(f"timed: {main_form['wall_ms']:.2f} ms/step; median Newton iteration {t_step:.2f} ms "
        f"(iterations {[round(x, 1) for x in main_form['iter_ms']]} ms, Krylov its {main_form['krylov_its']}), "
        f"adjoint {t_grad:.2f} ms ({main_form['adjoint_krylov_its']} its, {main_form['adjoint_sweeps']} sweeps)")
    vb = 8 if prec == fem.PREC_FP64 else 4
    avg_spmv_ms = main_form["spmv_ms"] / max(main_form["spmv_calls"], 1)
    nbytes = spmv_bytes(prob, vb, 8 if prec != fem.PREC_MIXED else 4)
    achieved = nbytes / (avg_spmv_ms * 1e-3) / 1e9
    log(f"SpMV: {main_form['spmv_calls']} timed launches, avg {avg_spmv_ms * 1e3:.1f} us, {achieved:.0f} GB/s")
    kname = "k_spmv_nodes (Krylov SpMV + FP64 dot)"
    prof_name = f"k_spmv_nodes_{p.name.replace('-', '_')}_{args.precision}_{args.krylov}.md"
    form_name = f"{args.precision} {args.precond}-{args.krylov}"
    out = {
        "metric": METRIC, "value": t_step + t_grad, "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main_form["wall_ms"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None,
        "dtype": {fem.PREC_MIXED: "f32 tangent/SpMV/Krylov + f64 residual/dots",
                  fem.PREC_MIXED_V64: "f32 tangent values + f64 Krylov vectors/SpMV arithmetic/residual",
                  fem.PREC_FP64: "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": (f"neo-Hookean tensile block {nx}x{ny}x{nz} HEX8 ({p.n_elems} elements, {p.n_dofs} "
                                f"dofs, nnz {prob.nnz}), lognormal G (ln 10, 0.3), kappa = 10 G, load step 5 of 5 to "
                                f"stretch 1.2" if u_obs is None else
                                f"inverse neo-Hookean block {nx}x{ny}x{nz} HEX8 on 2x1x1 ({p.n_elems} elements, "
                                f"{p.n_dofs} dofs, nnz {prob.nnz}), theta = 10 uniform, misfit to the solution at a "
                                f"seeded smooth theta_true, load step 5 of 5 to stretch 1.2")
                   + f"; {args.precond}-{args.krylov} (inner rtol {args.krylov_rtol:g}"
                     + (f", FP64-refined sweeps of {refine_for(fem, prec, kry):g}" if refine_for(fem, prec, kry) else "")
                     + f"), adjoint rtol {adjoint_rtol_for(fem, kry, args.adjoint_rtol):g}",
                   "precision": args.precision, "krylov": f"{args.precond}-{args.krylov}", "parallelism": "single GPU"},
        "newton_step_ms": t_step, "adjoint_grad_ms": t_grad,
        "t_step_definition": "median wall time of the Newton iterations of load step 5 (each: FP64 residual, "
                             "tangent assembly, Jacobi extraction, Krylov solve to the inner tolerance, update, "
                             "new residual); each timed step solves load step 5 from the converged state of load "
                             "step 4 and takes the gradient at its solution",
        "newton_iteration_ms": main_form["iter_ms"], "lifted_iteration_ms": main_form["iter_ms"][0],
        "dofs_per_s": p.n_dofs / (t_step * 1e-3),
        "krylov_its": {"newton_iterations": main_form["krylov_its"], "adjoint": main_form["adjoint_krylov_its"],
                       "adjoint_sweeps": main_form["adjoint_sweeps"]},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic(prof_name, KRYLOV_SOURCES),
                     "avg_launch_us": avg_spmv_ms * 1e3, "launches": main_form["spmv_calls"],
                     "launch_sampling": "HIP events around the SpMVs of the middle Krylov iteration of every "
                                        "16-iteration check block, over the timed steps",
                     "bytes_per_launch": nbytes,
                     "bytes_definition": "nnz*v + nnz/9*4 (one int32 per 3x3 block) + (Nn+1)*8 + 3*N*w "
                                         "(v: bytes per stored value, w: per vector entry)"},
    }
    out["roofline_assembly"] = assembly_roofline(fem, prob, main_form["u5"])
    log(f"assembly: {out['roofline_assembly']['avg_launch_us']:.0f} us, frac {out['roofline_assembly']['frac']:.3f}")

    fp64_counts = None
    if not args.no_compare:
        u5 = main_form["u5"]
        dJdu = objective_grad(u5)
        g_ref, _, _ = prob.adjoint_vjp(u5, dJdu, opts=prob.opts(precision=fem.PREC_FP64, krylov=fem.CG,
                                                                krylov_rtol=1e-8, adjoint_rtol=1e-11),
                                       want_lambda=False)

        def gerr(g):
            return float(torch.linalg.norm(g - g_ref) / torch.linalg.norm(g_ref))

        out["grad_rel_err_vs_fp64"] = gerr(main_form["g"])

        def row(r):
            return {"newton_step_ms": r["t_step"], "adjoint_grad_ms": r["t_grad"],
                    "value_ms": r["t_step"] + r["t_grad"], "newton_iteration_ms": r["iter_ms"],
                    "krylov_its": {"newton_iterations": r["krylov_its"], "adjoint": r["adjoint_krylov_its"]},
                    "grad_rel_err_vs_fp64_ref": gerr(r["g"])}

        # the plain FP64 form of the same step (same Krylov method and tolerances)
        f = measure(fem.PREC_FP64, kry, pc, 2, 1)
        out["fp64_step"] = row(f)
        out["fp64_step"]["speedup_mixed_over_fp64"] = (f["t_step"] + f["t_grad"]) / (t_step + t_grad)
        fp64_counts = {"newton_krylov_its": f["median_iteration_krylov_its"],
                       "adjoint_krylov_its": f["adjoint_krylov_its"], "adjoint_sweeps": f["adjoint_sweeps"]}
        log(f"fp64 {args.krylov} step: {f['t_step']:.1f} + {f['t_grad']:.1f} ms, "
            f"speedup of mixed {out['fp64_step']['speedup_mixed_over_fp64']:.2f}x")
        other = (("mixed_f32_vectors_step", fem.PREC_MIXED, kry, fem.PRECOND_JACOBI),
                 ("cg_step", fem.PREC_MIXED, fem.CG, fem.PRECOND_JACOBI),
                 ("bicgstab_step", prec, fem.BICGSTAB, fem.PRECOND_JACOBI),
                 ("block_jacobi_step", prec, kry, fem.PRECOND_BLOCK_JACOBI),
                 ("two_level_step", fem.PREC_MIXED, fem.CG, fem.PRECOND_AMG))
        for key, pr, kr, pcn in other:
            if (pr, kr, pcn) == (prec, kry, pc):
                continue
            if pcn == fem.PRECOND_AMG:
                t0 = time.perf_counter()
                n_agg, n_cb = prob.amg_sizes()
                t_setup = time.perf_counter() - t0
            try:
                amg = pcn == fem.PRECOND_AMG  # bounded, so that a failing two-level solve ends within minutes
                r = measure(pr, kr, pcn, 2, 1, krylov_max_it=2000 if amg else 20000, newton_max_it=12 if amg else 50)
            except fem.FemError as e:  # recorded, not fatal: the other rows still run
                out[key] = {"error": str(e)}
                log(f"{key}: {e}")
                continue
            out[key] = row(r)
            out[key]["form"] = ({fem.PREC_FP64: "fp64 ", fem.PREC_MIXED: "mixed (FP32 vectors) ",
                                 fem.PREC_MIXED_V64: "mixed64 (FP64 vectors) "}[pr]
                                + {0: "jacobi", 1: "block-jacobi", 2: "two-level"}[pcn] + "-"
                                + ("cg" if kr == fem.CG else "bicgstab"))
            if pcn == fem.PRECOND_AMG:
                out[key].update({"aggregates": n_agg, "coarse_blocks": n_cb, "setup_s": t_setup})
            out[key]["speedup_over_main"] = (t_step + t_grad) / (r["t_step"] + r["t_grad"])
            log(f"{key}: {r['t_step']:.1f} + {r['t_grad']:.1f} ms (its {r['krylov_its']} / {r['adjoint_krylov_its']})")
        # full 5-step solves against a tight FP64 solution
        u_ref, _ = prob.newton_solve(opts=prob.opts(precision=fem.PREC_FP64, krylov=fem.CG, krylov_rtol=1e-8,
                                                    newton_rtol=1e-11))
        res = {}
        forms = (("mixed64-bicgstab", fem.PREC_MIXED_V64, fem.BICGSTAB, fem.PRECOND_JACOBI, 0.0),
                 ("mixed-bicgstab", fem.PREC_MIXED, fem.BICGSTAB, fem.PRECOND_JACOBI, 0.5),
                 ("mixed-bicgstab-one-solve-per-correction", fem.PREC_MIXED, fem.BICGSTAB, fem.PRECOND_JACOBI, 0.0),
                 ("mixed-cg", fem.PREC_MIXED, fem.CG, fem.PRECOND_JACOBI, 0.0),
                 ("fp64-bicgstab", fem.PREC_FP64, fem.BICGSTAB, fem.PRECOND_JACOBI, 0.0),
                 ("fp64-cg", fem.PREC_FP64, fem.CG, fem.PRECOND_JACOBI, 0.0),
                 ("mixed-cg-two-level", fem.PREC_MIXED, fem.CG, fem.PRECOND_AMG, 0.0))
        for name, pr, kr, pcn, rr in forms:
            if pcn == fem.PRECOND_AMG and "error" in out.get("two_level_step", {}):
                res[name] = {"skipped": "the two-level step above failed: " + out["two_level_step"]["error"]}
                log(f"full 5-step solve {name}: skipped (the two-level step failed)")
                continue
            o = prob.opts(precision=pr, krylov=kr, newton_rtol=1e-9, krylov_rtol=args.krylov_rtol, precond=pcn,
                          refine_rtol=rr, max_bisections=4,
                          krylov_max_it=2000 if pcn == fem.PRECOND_AMG else 20000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                u, st = prob.newton_solve(opts=o)
            except fem.FemError as e:
                res[name] = {"error": str(e), "refine_rtol": rr}
                log(f"full 5-step solve {name}: {e}")
                continue
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            err = float(torch.linalg.norm(u - u_ref) / torch.linalg.norm(u_ref))
            res[name] = {"s": dt, "newton_its": st.newton_its, "krylov_its": st.krylov_its_total,
                         "rel_err_vs_tight_fp64": err, "refine_rtol": rr, "bisections": st.bisections}
            log(f"full 5-step solve {name}: {dt:.2f}s newton_its={st.newton_its} krylov_its={st.krylov_its_total} "
                f"err={err:.2e}")
        for a, b in (("fp64-bicgstab", "mixed64-bicgstab"), ("fp64-bicgstab", "mixed-bicgstab"),
                     ("fp64-cg", "mixed-cg")):
            if "s" in res[a] and "s" in res[b]:
                res[f"speedup_{b}_over_{a}".replace("-", "_")] = res[a]["s"] / res[b]["s"]
        out["full_solve"] = res
        if u_obs is None:
            next_rows(fem, inputs, out)

    prob.close()
    if not args.no_cpu_baseline and u_obs is None:
        if fp64_counts is None:  # without the comparison, the mixed form's counts stand in
            fp64_counts = {"newton_krylov_its": main_form["median_iteration_krylov_its"],
                           "adjoint_krylov_its": main_form["adjoint_krylov_its"],
                           "adjoint_sweeps": main_form["adjoint_sweeps"]}
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(fp64_counts, args.krylov)
        log(f"cpu baseline {time.perf_counter() - t0:.1f}s: {out['cpu_baseline']['value']:.0f} ms")
    for k in ("u5", "g"):
        main_form.pop(k, None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
