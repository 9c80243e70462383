"""Benchmark: line-DG residual+Jacobian throughput and BDF2 Newton-step time on one MI355X.

Workload (the 3-D Navier-Stokes headline configuration): Taylor-Green initial
data, M = 0.2, Re = 1600, Pr = 0.72, 32^3 hexes of [0, 2pi]^3 curved by
x + 0.1 sin x sin y sin z, p = 4 (125 nodes, 5 variables per element:
20.48 M unknowns), one BDF2 Newton step with dt = 0.02 from U^n = U^{n-1} = U0.

A step is one full Newton step of the chosen form: FP64 residual, FP64
Jacobian blocks stored in BF16, BF16 line-block ILU(0) (stored entries widened
to FP64 inside the products), GMRES(50) wrapped in FP64 iterative refinement
with the exact tangent product until ||b - (I - gamma A) dU|| <= 1e-8 ||b||.  The plain FP64 step (FP64
blocks and factors, GMRES to 1e-8 directly) is timed beside it.

value = residual+Jacobian DOF/s = DOFs / (t_residual + t_assembly), both
measured with HIP events inside the timed Newton steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C4", choices=["C3", "C4"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=256, help="elements timed on the CPU oracle")
    ap.add_argument("--no-rk4", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 16^3, DIRK3 and 512^2 measurements")
    ap.add_argument("--coupled-only", action="store_true",
                    help="run only the coupled C22 solve measurement and print its record (for profiling)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy 1 GiB between two device buffers first (a reference kernel for profiler counters)")
    return ap.parse_args()


HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "solver_kernels_tgv32p4_bf16_traffic.md")
TRAFFIC_SOURCE = {"jacvec": "k_precond.hip", "precond_apply": "k_precond.hip", "k21_product": "k_k21.hip"}


def measured_traffic(kernel):
    """HBM bytes per launch of one solver kernel from the committed rocprofv3 counter summary.

    The summary records FETCH_SIZE / WRITE_SIZE per dispatch, each scaled by what the same counter
    reads for a plain copy kernel of known size, and the SHA-256 of the kernel's source file it was
    taken with; a changed source makes the figure stale, and then None is reported.
    """
    import hashlib
    import re
    if not os.path.exists(TRAFFIC_FILE) or kernel not in TRAFFIC_SOURCE:
        return None
    txt = open(TRAFFIC_FILE).read()
    m_b = re.search(r"traffic_bytes_per_launch\[" + kernel + r"\]\s*=\s*([0-9.eE+]+)", txt)
    fname = TRAFFIC_SOURCE[kernel]
    m_h = re.search(r"source_sha256\[" + re.escape(fname) + r"\]\s*=\s*([0-9a-f]{64})", txt)
    if not m_b or not m_h:
        return None
    src = os.path.join(ROOT, "paper_1204_1533_amd", "csrc", fname)
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_h.group(1):
        return None
    return float(m_b.group(1))


def roofline(pr, reps, prec):
    """Achieved bandwidth of the solver's stream-timed kernels (HIP events inside the step).

    Algorithmic bytes per node (m components, D dimensions, p degree, e bytes per stored entry):
      split product: K11 (Dp+1+2D) m^2 e + K12 (Dp+1+D) m^2 D e + x 8m + w = K21 x 8mD + y 8m
      ILU(0) apply : factors (Dp+1) m^2 e + r 8m + z 8m
      K21 x        : stored weights (Dp+1+D) D ew + x 8m + w 8mD, ew = 4 (FP32 copy) in the products
                     with stored FP32 / BF16 blocks, 8 in the refinement's exact products and with
                     FP64 storage; the per-launch figure averages the step's launches of both
    """
    import numpy as np
    me = pr.mesh
    D, p, m = me.dim, me.p, pr.m
    e = {0: 8, 1: 4, 2: 2}[prec]
    nodes = me.n_elem * me.np_
    per_node = {
        "jacvec": (D * p + 1 + 2 * D) * m * m * e + (D * p + 1 + D) * m * m * D * e + 8 * m + 8 * m * D + 8 * m,
        "precond_apply": (D * p + 1) * m * m * e + 16 * m,
        "k21_product": None,
    }
    k21_f64 = (D * p + 1 + D) * D * 8 + 8 * m + 8 * m * D
    k21_stored = (D * p + 1 + D) * D * (8 if prec == 0 else 4) + 8 * m + 8 * m * D
    keys = {"jacvec": ("t_jacvec_ms", "n_jacvec"), "precond_apply": ("t_precond_ms", "n_precond"),
            "k21_product": ("t_k21_ms", "n_k21")}
    allk = {}
    for k, (tk, nk) in keys.items():
        tot = float(np.sum([r[tk] for r in reps]))
        n = int(np.sum([r[nk] for r in reps]))
        if n == 0:
            continue
        avg_ms = tot / n
        if k == "k21_product":
            n_stored = min(n, int(np.sum([r["n_jacvec"] for r in reps])))
            byts = (n_stored * k21_stored + (n - n_stored) * k21_f64) / n * nodes
        else:
            byts = per_node[k] * nodes
        gbs = byts / (avg_ms * 1e-3) / 1e9
        allk[k] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                   "traffic": None, "avg_ms": avg_ms, "launches": n, "bytes_per_launch": byts,
                   "share_of_step_ms": tot / len(reps)}
    dom = max(allk, key=lambda k: allk[k]["share_of_step_ms"]) if allk else None
    if prec == 2 and me.n_elem == 32768 and p == 4:
        for k in allk:
            allk[k]["traffic"] = measured_traffic(k)
    d = dict(allk[dom]) if dom else None
    if d:
        d["kernel"] = dom
    return {"dominant": d, "all": allk}


FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
FLOPS_FILE = os.path.join(ROOT, "profiles", "residual_tgv32p4_fp64_flops.md")


def counted_residual_flops():
    """FP64 operations of one residual evaluation (gradient + residual kernels) from the committed
    rocprofv3 VALU instruction counts, or None when the kernel source has changed since."""
    import hashlib
    import re
    if not os.path.exists(FLOPS_FILE):
        return None
    txt = open(FLOPS_FILE).read()
    m_f = re.search(r"residual_flops_per_eval\s*=\s*([0-9.eE+]+)", txt)
    m_h = re.search(r"source_sha256\s*=\s*([0-9a-f]{64})", txt)
    if not m_f or not m_h:
        return None
    src = os.path.join(ROOT, "paper_1204_1533_amd", "csrc", "k_resid.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_h.group(1):
        return None
    return float(m_f.group(1))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pr, n_sample, gmres_iters, refine_sweeps):
    """The FP64 CPU oracle timed on bounded samples of the workload (about half a minute in all).

    All host threads: residual (median of 3) and Jacobian blocks of n_sample seeded elements of the
    32^3 p=4 workload; the split product, the A~ formation + BILU(0) factorisation and the BILU(0)
    apply on the 2^3 p=4 mesh of the same equations (medians of 5, scaled per unknown).  One
    thread: residual and Jacobian blocks of n_sample/8 elements.  The oracle Newton step on the
    workload is estimated from these per-unknown costs and the GPU step's iteration counts."""
    import numpy as np
    import torch
    from ldg_workloads import configs
    from oracle import LineDG, Physics, solver

    def disc(p_):
        me = p_.mesh
        ph = Physics(p_.equation, me.dim, gamma=p_.gamma, mu=p_.mu, prandtl=p_.prandtl)
        return LineDG(me.dim, me.p, me.xyz, me.face_nbr, me.nbr_node, me.switch_plus, ph, p_.c11_interior,
                      p_.c11_dirichlet, p_.source, p_.gD)

    def med(fn, k):
        ts = []
        for _ in range(k):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    me = pr.mesh
    dof_el = pr.m * me.np_
    orc = disc(pr)
    rng = np.random.default_rng(0)
    el = np.sort(rng.choice(me.n_elem, size=min(n_sample, me.n_elem), replace=False))
    threads = torch.get_num_threads()
    orc.residual(pr.U0, elems=el[:2])  # warm-up
    t_res = med(lambda: orc.residual(pr.U0, elems=el), 3)
    t_jac = med(lambda: orc.jacobian(pr.U0, elems=el), 1)
    # split product, formation + factorisation, apply on the 2^3 mesh of the same equations
    small = configs.taylor_green(2, me.p, pr.extra.get("re", 1600.0), dt=pr.dt)
    os_ = disc(small)
    K11, K12, K21 = os_.jacobian(small.U0)
    gamma = 2.0 * pr.dt / 3.0
    x = torch.randn(os_.E, os_.m, os_.Np, dtype=torch.float64, generator=torch.Generator().manual_seed(0))
    c11, c12 = os_.column_nodes("K11"), os_.column_nodes("K12")
    pat = solver.line_pattern(os_)
    t_mv = med(lambda: solver.split_matvec(os_, K11, K12, x, gamma, 1.0, c11, c12), 5)
    holder = {}

    def form_factor():
        holder["F"] = solver.bilu0(solver.precond_matrix(os_, K11, K12, K21, gamma, 1.0), pat)

    t_ff = med(form_factor, 1)
    t_ap = med(lambda: solver.bilu0_apply(holder["F"], pat, x), 5)
    small_dofs = small.n_dof
    # one thread
    torch.set_num_threads(1)
    try:
        el1 = el[: max(1, len(el) // 8)]
        t_res1 = med(lambda: orc.residual(pr.U0, elems=el1), 1)
        t_jac1 = med(lambda: orc.jacobian(pr.U0, elems=el1), 1)
    finally:
        torch.set_num_threads(threads)
    dofs = len(el) * dof_el
    dofs1 = len(el1) * dof_el
    per = {"residual_s_per_mdof": t_res / dofs * 1e6, "jacobian_s_per_mdof": t_jac / dofs * 1e6,
           "split_product_s_per_mdof": t_mv / small_dofs * 1e6,
           "precond_form_factor_s_per_mdof": t_ff / small_dofs * 1e6,
           "precond_apply_s_per_mdof": t_ap / small_dofs * 1e6}
    N = pr.n_dof
    # a Newton step: residuals (start, end, one per refinement sweep for the exact tangent is
    # counted as a split product), assembly, formation + factorisation, GMRES iterations
    est = (2 * t_res / dofs + t_jac / dofs + t_ff / small_dofs
           + (gmres_iters + refine_sweeps) * (t_mv + t_ap) / small_dofs) * N
    log(f"[bench] cpu oracle ({threads} threads): residual {t_res:.2f} s + Jacobian {t_jac:.2f} s for "
        f"{len(el)} elements; 1 thread {t_res1 + t_jac1:.2f} s for {len(el1)}")
    return {"value": dofs / (t_res + t_jac), "unit": "DOF/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"residual (median of 3) + Jacobian blocks (K11, K12) of {len(el)} seeded elements of the "
                      f"workload with {threads} threads ({t_res + t_jac:.1f} s); split product, A~ formation + "
                      f"BILU(0) and apply on the 2^3 p={me.p} mesh of the same equations, per unknown",
            "single_core": {"value": dofs1 / (t_res1 + t_jac1), "unit": "DOF/s", "cores": 1,
                            "sample": f"residual + Jacobian blocks of {len(el1)} elements"},
            "per_op": per,
            "newton_step_estimate_s": est,
            "newton_step_estimate_note": "per-unknown oracle costs x the workload's unknowns, with the GPU "
                                         "chosen step's GMRES iterations and refinement sweeps"}


def rk4_c2(Context):
    """Explicit RK4 on the 2-D Euler vortex (32^2 perturbed quads, p=4, 102 k unknowns): each step
    replays a captured graph of the 4 residual evaluations and stage updates."""
    import torch
    from ldg_workloads import configs
    pr = configs.config2()
    ctx = Context(pr.mesh, pr.equation, gamma=pr.gamma, stream=torch.cuda.current_stream().cuda_stream)
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    ctx.ldg_rk4(U, pr.dt, 10)
    torch.cuda.synchronize()
    n = 100
    t0 = time.perf_counter()
    ctx.ldg_rk4(U, pr.dt, n)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / n
    ctx.close()
    log(f"[bench] C2 RK4: {ms:.3f} ms per step")
    # per step: 4 residual launches, 4 stage updates and 2 copies (10 kernels) replayed from a graph;
    # the 0.8 MB state stays in the caches, so the step is bound by the kernels' latency, not by HBM
    return {"workload": "2-D Euler isentropic vortex, 32x32 perturbed quads, p=4, 102400 unknowns",
            "dt": pr.dt, "steps": n, "ms_per_step": ms, "residual_evals_dof_per_s": pr.n_dof * 4 / (ms * 1e-3),
            "kernels_per_step": 10, "us_per_kernel": ms * 1e3 / 10,
            "bound": "launch latency (graph replay of 10 dependent kernels on a cache-resident 0.8 MB state)"}


def c3_newton(Context):
    """The 16^3 p=3 Navier-Stokes workload (1.31 M unknowns): one BDF2 Newton step in its chosen form
    (FP32 blocks and factors, FP64 refinement) and in plain FP64, after a warm-up step each; both
    again with the exact element-block LU preconditioner in place of BILU(0)."""
    import numpy as np
    import torch
    from ldg_workloads import configs
    from paper_1204_1533_amd import LDG_F32, LDG_F64
    pr = configs.config3()
    ctx = Context(pr.mesh, pr.equation, gamma=pr.gamma, mu=pr.mu, prandtl=pr.prandtl,
                  stream=torch.cuda.current_stream().cuda_stream)
    U0 = torch.as_tensor(pr.U0, device="cuda").contiguous()
    U = U0.clone()
    gamma = 2.0 * pr.dt / 3.0
    out = {"workload": f"{pr.name}: 16^3 hexes, p=3, Re=400, BDF2 dt={pr.dt}, {pr.n_dof} unknowns"}
    res = {}
    from paper_1204_1533_amd.ldg import LDG_PRECOND_BILU0, LDG_PRECOND_BLOCK_LU
    for name, prec, inner, kind in (("chosen_fp32", LDG_F32, 0.15, LDG_PRECOND_BILU0),
                                    ("plain_fp64", LDG_F64, 1e-3, LDG_PRECOND_BILU0),
                                    ("block_lu_fp32", LDG_F32, 0.15, LDG_PRECOND_BLOCK_LU),
                                    ("block_lu_fp64", LDG_F64, 1e-3, LDG_PRECOND_BLOCK_LU)):
        ctx.ldg_set_preconditioner(kind)
        reps = []
        for k in range(2):
            U.copy_(U0)
            reps.append(ctx.ldg_newton_step(U, U0, 1.0, gamma, storage_prec=prec, restart=50, max_iters=2000,
                                            max_refine=40, rtol=1e-8, inner_rtol=inner))
        r = reps[-1]
        res[name] = U - U0
        out[name] = {"ms_per_step": r["t_total_ms"], "gmres_iters": r["gmres_iters"],
                     "refine_steps": r["refine_steps"], "lin_relres": r["lin_relres"],
                     "t_resid_ms": r["t_resid_ms"], "t_assemble_ms": r["t_assemble_ms"],
                     "t_solve_ms": r["t_solve_ms"],
                     "residual_jacobian_dof_per_s": pr.n_dof / ((r["t_resid_ms"] + r["t_assemble_ms"]) * 1e-3)}
        log(f"[bench] C3 {name}: {r['t_total_ms']:.1f} ms, gmres {r['gmres_iters']}")
    d = res["chosen_fp32"] - res["plain_fp64"]
    out["dU_max_diff_rel"] = float(d.abs().max() / res["plain_fp64"].abs().max())
    d = res["block_lu_fp64"] - res["plain_fp64"]
    out["dU_max_diff_rel_block_lu"] = float(d.abs().max() / res["plain_fp64"].abs().max())
    out["block_lu_note"] = ("exact element-block LU of A~ (dense 320 x 320 per element, FP64) in place of "
                            "BILU(0); same Newton step, GMRES iterations and times for comparison")
    ctx.close()
    return out


def dirk3_reuse_c3(Context):
    """One DIRK3 step (Section 4.1) on the 16^3 p=3 workload with 5 GMRES iterations per Newton
    iteration (FP32 blocks), with the Jacobian re-used across Newton iterations and stages
    (re-assembled after 15 Newton iterations of a stage, Section 4.3) and with a fresh Jacobian at
    every Newton iteration; stage tolerance 1e-8 of the stage's starting ||G||."""
    import torch
    from ldg_workloads import configs
    from paper_1204_1533_amd import LDG_F32
    from paper_1204_1533_amd.ldg import LDG_DIRK3
    pr = configs.config3()
    ctx = Context(pr.mesh, pr.equation, gamma=pr.gamma, mu=pr.mu, prandtl=pr.prandtl,
                  stream=torch.cuda.current_stream().cuda_stream)
    U0 = torch.as_tensor(pr.U0, device="cuda").contiguous()
    out = {"workload": f"{pr.name}, DIRK3 dt={pr.dt}, 5 GMRES iterations per Newton iteration, FP32 blocks"}
    res = {}
    for name, reuse in (("reuse", 1), ("fresh", 0)):
        U = U0.clone()
        r = ctx.ldg_implicit_step(U, None, pr.dt, scheme=LDG_DIRK3, max_newton=80, newton_rtol=1e-8, reuse=reuse,
                                  reassemble_after=15, gmres_per_newton=5, storage_prec=LDG_F32, raise_on_error=False)
        res[name] = U
        out[name] = {k: r[k] for k in ("t_ms", "newton_iters", "max_stage_newton", "assemblies", "gmres_iters",
                                       "converged", "newton_res_final", "t_assemble_ms", "t_solve_ms")}
        log(f"[bench] C3 DIRK3 {name}: {r['t_ms']:.1f} ms, newton {r['newton_iters']}, "
            f"assemblies {r['assemblies']}")
    out["U_max_diff_rel"] = float((res["reuse"] - res["fresh"]).abs().max() / (res["fresh"] - U0).abs().max())
    ctx.close()
    return out


def euler_residual_bandwidth(Context):
    """FP64 Euler residual on the tiled vortex, 512^2 perturbed quads at p=4 (26.2 M unknowns):
    median time of 20 evaluations against the HBM roof of its algorithmic bytes (state read,
    residual written: 8m + 8m per node, plus each element's geometry record of
    D NL NG D + D 2NL D + Np doubles) and the FP64 roof."""
    import numpy as np
    import torch
    from ldg_workloads import configs
    pr = configs.euler_vortex_tiled(512, 4)
    ctx = Context(pr.mesh, pr.equation, gamma=pr.gamma, stream=torch.cuda.current_stream().cuda_stream)
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    R = torch.empty_like(U)
    for _ in range(3):
        ctx.ldg_residual(U, R)
    torch.cuda.synchronize()
    ts = []
    for _ in range(20):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ctx.ldg_residual(U, R)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ms = float(np.median(ts))
    nodes = pr.mesh.n_elem * pr.mesh.np_
    D, n1 = pr.mesh.dim, pr.mesh.p + 1
    ng = (3 * pr.mesh.p + 2) // 2  # Gauss points per line: ceil((3p + 1) / 2)
    nl = n1 ** (D - 1)
    rec = D * nl * ng * D + D * 2 * nl * D + pr.mesh.np_
    byts = nodes * (8 * pr.m + 8 * pr.m) + pr.mesh.n_elem * rec * 8
    gbs = byts / (ms * 1e-3) / 1e9
    ctx.close()
    log(f"[bench] 512^2 Euler residual: {ms:.3f} ms, {gbs:.0f} GB/s algorithmic")
    return {"workload": f"{pr.name}: {pr.n_dof} unknowns", "ms_per_residual": ms,
            "dof_per_s": pr.n_dof / (ms * 1e-3), "bytes_per_eval": byts, "achieved_gbs": gbs,
            "frac_hbm": gbs / HBM_PEAK_GBS}


def coupled_poisson(Context):
    """Steady coupled (U, Q) solve with C11 = C22 = 1/20 (Section 4.1; the scheme of Table poitab1's
    second block) on 16^2 perturbed quads, p = 3, next to the reduced system (C22 = 0) solved by one
    steady Newton step: wall time, outer and inner iterations.  Steady elliptic solves with the
    element-local preconditioner need iteration counts that grow with the mesh (no global
    coarse correction; the paper solves these systems with a sparse direct solver), which keeps
    this measurement small."""
    import time
    import torch
    from ldg_workloads import configs, fields, quad_mesh
    mesh = quad_mesh(16, 16, 3, box=((0, 1), (0, 1)), perturb=0.2, seed=2)
    u, f, g = fields.poisson_sine(mesh)
    pr = configs.Problem("poisson16p3_pert", mesh, configs.EQ_POISSON, 1, 0 * u, c11_interior=1 / 20, source=f,
                         gD=fields.face_values(mesh, u))
    ctx = Context(pr.mesh, pr.equation, c11_interior=pr.c11_interior, c11_dirichlet=pr.c11_dirichlet,
                  stream=torch.cuda.current_stream().cuda_stream)
    S = torch.as_tensor(pr.source, device="cuda").contiguous()
    gD = torch.as_tensor(pr.gD, device="cuda").contiguous()
    ctx.ldg_set_source(S)
    ctx.ldg_set_dirichlet(gD)
    E, Np = mesh.n_elem, mesh.np_
    U = torch.zeros(E, 1, Np, dtype=torch.float64, device="cuda")
    Q = torch.zeros(E, 1, 2, Np, dtype=torch.float64, device="cuda")
    out = {"workload": f"{pr.name}: {E * Np} + {2 * E * Np} unknowns (U, Q), C11 = C22 = 1/20"}
    ctx.ldg_set_c22(1 / 20)
    kw = dict(rtol=1e-10, inner_rtol=1e-3, restart=60, max_iters=500, raise_on_error=False)
    ctx.ldg_coupled_solve(U, Q, **kw)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.ldg_coupled_solve(U, Q, **kw)
    torch.cuda.synchronize()
    out["coupled"] = {"ms": 1e3 * (time.perf_counter() - t0), "status": r["status"], "outer_iters": r["iters"],
                      "inner_iters": r["inner_iters"], "relres": r["relres"],
                      "q_err_max": float((Q.cpu() - torch.as_tensor(g)).abs().max())}
    ctx.ldg_set_c22(0.0)
    U.zero_()
    ctx.ldg_newton_step(U, U.clone(), 0.0, 1.0, restart=60, max_iters=3000, rtol=1e-10, raise_on_error=False)
    U.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rr = ctx.ldg_newton_step(U, U.clone(), 0.0, 1.0, restart=60, max_iters=3000, rtol=1e-10, raise_on_error=False)
    torch.cuda.synchronize()
    ctx.ldg_gradient(U, Q)
    torch.cuda.synchronize()
    out["reduced_c22_0"] = {"ms": 1e3 * (time.perf_counter() - t0), "gmres_iters": rr["gmres_iters"],
                            "lin_relres": rr["lin_relres"],
                            "q_err_max": float((Q.cpu() - torch.as_tensor(g)).abs().max())}
    ctx.close()
    log(f"[bench] coupled C22 solve: {out['coupled']['ms']:.1f} ms ({r['iters']} outer, {r['inner_iters']} inner); "
        f"reduced {out['reduced_c22_0']['ms']:.1f} ms")
    return out


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only: sharding the elements over several GPUs is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from ldg_workloads import configs
    from paper_1204_1533_amd import Context, LDG_BF16, LDG_F64, LDG_F32

    torch.cuda.set_device(0)
    if args.coupled_only:
        print(json.dumps({"coupled_c22": coupled_poisson(Context)}))
        return
    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    pr = configs.config4() if args.config == "C4" else configs.config3()
    chosen_prec = LDG_BF16 if args.config == "C4" else LDG_F32
    log(f"[bench] workload {pr.name}: E={pr.mesh.n_elem} p={pr.mesh.p} dofs={pr.n_dof}")
    stream = torch.cuda.current_stream().cuda_stream
    ctx = Context(pr.mesh, pr.equation, gamma=pr.gamma, mu=pr.mu, prandtl=pr.prandtl, stream=stream)
    U0 = torch.as_tensor(pr.U0, device="cuda").contiguous()
    U = U0.clone()
    gamma = 2.0 * pr.dt / 3.0
    # inner tolerance of each refinement sweep: the BF16 operator limits what one sweep can gain,
    # so loose sweeps (0.15, measured best among 1e-4 .. 0.5) waste the fewest GMRES iterations
    opts = dict(restart=50, max_iters=2000, max_refine=40, rtol=1e-8, inner_rtol=0.15, reassemble=1)

    def step(prec):
        U.copy_(U0)
        return ctx.ldg_newton_step(U, U0, 1.0, gamma, storage_prec=prec, **opts)

    for _ in range(args.warmup):
        step(chosen_prec)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        reps.append(step(chosen_prec))
        log(f"[bench] chosen step {k}: {reps[-1]['t_total_ms']:.1f} ms, gmres {reps[-1]['gmres_iters']}, "
            f"refine {reps[-1]['refine_steps']}, relres {reps[-1]['lin_relres']:.2e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    t_res = float(np.mean([r["t_resid_ms"] for r in reps]))
    t_asm = float(np.mean([r["t_assemble_ms"] for r in reps]))
    value = pr.n_dof / ((t_res + t_asm) * 1e-3)
    U_chosen = U.clone()

    plain = None
    if not args.no_plain:
        r = step(LDG_F64)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        prs = []
        for k in range(max(1, args.steps // 2)):
            prs.append(step(LDG_F64))
            log(f"[bench] plain fp64 step {k}: {prs[-1]['t_total_ms']:.1f} ms, gmres {prs[-1]['gmres_iters']}")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        plain = dict(ms_per_step=(t3 - t2) * 1e3 / len(prs), gmres_iters=prs[-1]["gmres_iters"],
                     lin_relres=prs[-1]["lin_relres"], newton_res_after=prs[-1]["newton_res_after"],
                     t_resid_ms=float(np.mean([p["t_resid_ms"] for p in prs])),
                     t_assemble_ms=float(np.mean([p["t_assemble_ms"] for p in prs])),
                     t_solve_ms=float(np.mean([p["t_solve_ms"] for p in prs])),
                     dU_max_diff_rel=float((U - U_chosen).abs().max() / (U - U0).abs().max()))

    rk4 = rk4_c2(Context) if not args.no_rk4 else None
    extra = None
    if not args.no_extra:
        extra = {"c3_newton": c3_newton(Context), "dirk3_c3": dirk3_reuse_c3(Context),
                 "euler_residual_512": euler_residual_bandwidth(Context), "coupled_c22": coupled_poisson(Context)}
    last = reps[-1]
    roof = roofline(pr, reps, chosen_prec)
    # residual (gradient + residual kernels) against the FP64 roof with algorithmic operations:
    # about 880 FLOP per unknown for the 3-D p=4 Navier-Stokes residual (operation count of the
    # algorithm: flux evaluations at the D (p+1)^2 n_g Gauss points and 2D (p+1)^2 face points,
    # the (p+1) x n_g line contractions, Roe solves), counted FP64 operations beside it
    alg = 880.0 * pr.n_dof if (pr.mesh.dim == 3 and pr.mesh.p == 4) else None
    if alg is not None:
        tf = alg / (t_res * 1e-3) / 1e12
        fl = counted_residual_flops() if pr.mesh.n_elem == 32768 else None
        roof["all"]["residual"] = {"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": tf / FP64_PEAK_TFLOPS, "avg_ms": t_res, "flops_per_eval": alg,
                                   "counted_flops_per_eval": fl,
                                   "note": "algorithmic FP64 operations (880 per unknown) over the stream-timed "
                                           "gradient + residual kernels"}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pr, args.cpu_sample, last["gmres_iters"], last["refine_steps"])
    out = {
        "metric": "residual+Jacobian DOF/s; Newton step time to 1e-8, plain FP64 vs chosen form",
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{pr.name}: 3-D Navier-Stokes Taylor-Green, Re={pr.extra['re']:.0f}, "
                               f"M=0.2, p={pr.mesh.p}, {pr.mesh.n_elem} hexes, BDF2 dt={pr.dt}",
                   "dofs": pr.n_dof,
                   "storage_prec": {0: "f64", 1: "f32", 2: "bf16"}[chosen_prec]},
        "newton": {"chosen": {"ms_per_step": ms_step, "gmres_iters": last["gmres_iters"],
                              "refine_steps": last["refine_steps"], "lin_relres": last["lin_relres"],
                              "newton_res_before": last["newton_res_before"],
                              "newton_res_after": last["newton_res_after"],
                              "t_resid_ms": t_res, "t_assemble_ms": t_asm,
                              "t_solve_ms": float(np.mean([r["t_solve_ms"] for r in reps]))},
                   "plain_fp64": plain},
        "roofline": roof["dominant"],
        "kernels": roof["all"],
        "cpu_baseline": cpu,
        "rk4_c2": rk4,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
