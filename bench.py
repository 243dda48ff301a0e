"""Benchmark: factor+solve DOF/s of the slab solver on one MI355X.

Workload: -div(kappa grad u) = f on 2048 rows x 4096 columns (8.39M unknowns),
slab width b = 31 (128 slabs, interfaces of 2048 points), kappa = exp(GRF)
(squared-exponential covariance, length 0.05, variance 1), 16 right-hand sides
N(0,1).  One step = slab_factor + slab_solve of all 16 right-hand sides to a
max relative residual of 1e-10 + slab_free.  The headline value is the
mixed form (FP64 slab work, FP32 reduced system, FP64 refinement) with stage
two in odd-even order; the all-FP32 form, the sweep of Alg. 1 and the plain
FP64 form are timed beside it.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from gen import inputs as G  # noqa: E402

HBM_PEAK_GBS = 8000.0


def finite_json(obj):
    """obj with every non-finite float replaced by None (strict JSON)."""
    if isinstance(obj, dict):
        return {k: finite_json(v) for k, v in obj.items()}
    if isinstance(obj, (list, tuple)):
        return [finite_json(v) for v in obj]
    if isinstance(obj, float) and not np.isfinite(obj):
        return None
    return obj


def log(msg: str) -> None:
    """Progress line on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)

PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diffusion_2048x4096_b31",
                    help="diffusion_2048x4096_b31 (headline), diffusion_1024x1024_b31, "
                         "poisson_64x64_b7, adjoint_512x512_b15 or batch256")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--precision", choices=["mixed", "fp32"], default="mixed",
                    help="mixed: FP64 slab work + FP32 reduced system; fp32: FP32 throughout "
                         "(both with FP64 refinement to 1e-10)")
    ap.add_argument("--order", choices=["odd_even", "sweep"], default="odd_even",
                    help="stage two: odd-even elimination order or the sweep of Alg. 1")
    ap.add_argument("--skip-other", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy (scales the HBM counters)")
    ap.add_argument("--autotune", action="store_true",
                    help="also report the slab width the autotuner picks for the grid")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-extra", action="store_true",
                    help="skip the 1024x1024 and 512x512 lines")
    ap.add_argument("--cpu-slabs", type=int, default=1)
    return ap.parse_args()


def run_batch(warmup: int, steps: int) -> dict:
    """The batch of 256 uneven problems (grid sides n2 in {128..1024}, n1 in
    {128..2048}, b in {7,15,31}, 1-16 uniform right-hand sides, lognormal
    kappa; mixed precision, odd-even order, refinement to 1e-10 with at most
    3 passes).  Setup (untimed): slab_factor_batch allocates and factors once.
    A step is slab_batch_run: the factorization of all 256 problems and all
    refinement passes of their solves as one HIP graph launch (captured in the
    first warm-up step), reading the coefficient fields and loads from the
    same device buffers.  The eager form (slab_factor_batch +
    slab_solve_batch + slab_batch_free per step) is timed beside it."""
    import torch
    from paper_2211_07572_amd import slab as S
    probs = G.batch_problems(256)
    t0 = time.perf_counter()
    kaps = [torch.as_tensor(w.kappa(), device="cuda") for w in probs]
    fs = [torch.as_tensor(w.rhs(), device="cuda") for w in probs]
    gen_s = time.perf_counter() - t0
    dims = [(w.n2, w.n1, w.b) for w in probs]
    torch.cuda.synchronize()
    opts = dict(precision=S.SLAB_MIXED, tol=1e-10, max_iter=3, odd_even=True)
    t0 = time.perf_counter()
    bt = S.slab_factor_batch(kaps, dims, graph=True, **opts)
    setup_s = time.perf_counter() - t0
    outs = [torch.empty_like(f) for f in fs]
    times, infos = [], []
    for it in range(max(warmup, 1) + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.slab_batch_run(bt, kaps, fs, outs=outs)   # synchronizes once, at its end
        dt = time.perf_counter() - t0
        if it >= max(warmup, 1):
            times.append(dt)
            infos.append([(i.iterations, i.max_relres) for i in bt.last_infos])
    bt.free()
    # eager form, one warm-up and `steps` timed steps
    eager = []
    for it in range(1 + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b2 = S.slab_factor_batch(kaps, dims, **opts)
        S.slab_solve_batch(b2, fs, outs=outs)
        b2.free()
        torch.cuda.synchronize()
        if it >= 1:
            eager.append(time.perf_counter() - t0)
    med = float(np.median(times))
    dof = sum(w.N for w in probs)
    return {"value": dof / med, "unit": "DOF/s", "ms_per_step": med * 1e3,
            "step_ms": [t * 1e3 for t in times], "steps": steps, "warmup": max(warmup, 1),
            "problems": len(probs), "dof": dof, "rhs_total": sum(w.nrhs for w in probs),
            "step": "slab_batch_run (factor + solve + up to 3 refinement passes, one graph launch)",
            "max_relres": max(r for step in infos for _, r in step),
            "max_refine_passes": max(i for step in infos for i, _ in step),
            "eager_ms_per_step": float(np.median(eager)) * 1e3,
            "setup_s": setup_s, "input_generation_s": gen_s}


def run_batch_line(args) -> dict:
    """--workload batch256: the batch as the JSON line's headline."""
    r = run_batch(args.warmup, args.steps)
    return {"metric": "factor+solve DOF/s, FP32+refine vs FP64 on GPU at rel. residual 1e-10",
            "value": r["value"], "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
            "warmup": r["warmup"], "ms_per_step": r["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "batch256_uneven", "problems": r["problems"], "dof": r["dof"],
                       "rhs_total": r["rhs_total"], "tol": 1e-10,
                       "precision": "FP64 slab work, FP32 reduced system, FP64 refinement",
                       "stage_two": "odd-even elimination order", "graph": True},
            "batch": r}


def workload(name: str) -> G.Workload:
    table = {w.name: w for w in (G.POISSON_64, G.DIFFUSION_1024, G.DIFFUSION_2048x4096, G.ADJOINT_512)}
    return table[name]


def schur_flops(w: G.Workload) -> float:
    """Algorithmic flops of the Schur propagation (one launch covers every slab):
    per slab 2n chains (n for slab 0), chain rho propagated over n-1-rho steps of
    a b x b matrix-vector product (2 b^2 flops)."""
    n, b, m = w.n2, w.b, w.m
    return 2.0 * b * b * n * (n - 1) * (m - 0.5)


def block_factor_flops(w: G.Workload, odd_even: bool) -> float:
    """Algorithmic flops of the block factorization.  Every pivot block: the
    Cholesky factor (n^3/3) and its inverse (n^3/3).  Alg. 1: per coupling
    Z_j = L_j^-1 T_{j,j+1} (n^3) and the symmetric update of S_{j+1} (n^3).
    Odd-even: per eliminated block with a neighbour before it U = L^-1 C^T (n^3)
    and D_l -= U^T U (n^3), likewise V and D_r with a neighbour after it, and
    the new coupling -U^T V (2n^3) with both."""
    n, m = w.n2, w.m
    if not odd_even:
        return m * (2.0 / 3.0) * n ** 3 + (m - 1) * 2.0 * n ** 3
    total, s = 0.0, 1
    while m // s >= 1:
        k = m // s
        E, NR = (k + 1) // 2, k // 2
        total += E * (2.0 / 3.0) * n ** 3 + (E - 1) * 2.0 * n ** 3 + NR * 2.0 * n ** 3
        total += max(NR - 1, 0) * 2.0 * n ** 3
        s *= 2
    return total


def block_products(w: G.Workload, odd_even: bool, elem: int = 4):
    """Launches of the block products of stage two (the GEMM kernel): total
    algorithmic flops, total algorithmic HBM bytes and the number of launches.
    Per item (n x n blocks): a product with a lower-triangular factor
    (L^-1 C: n^3 flops; reads n^2/2 + n^2, writes n^2), a symmetric update
    (D -= U^T U, lower half: n^3 flops; reads n^2 + n^2/2, writes n^2/2) and a
    full product (-U^T V: 2 n^3 flops; reads 2 n^2, writes n^2)."""
    n, m = w.n2, w.m
    n2, n3 = float(n) ** 2, float(n) ** 3
    tri = (n3, 2.5 * n2 * elem)
    sym = (n3, 2.0 * n2 * elem)
    full = (2 * n3, 3.0 * n2 * elem)
    fl = by = 0.0
    launches = 0

    def add(kind, count):
        nonlocal fl, by, launches
        if count > 0:
            fl += kind[0] * count
            by += kind[1] * count
            launches += 1
    if not odd_even:
        for j in range(m):
            add(sym, 1 if j > 0 else 0)
            add(tri, 1 if j < m - 1 else 0)
        return fl, by, launches
    s = 1
    while m // s >= 1:
        k = m // s
        E, NR = (k + 1) // 2, k // 2
        add(tri, E - 1)
        add(tri, NR)
        add(sym, E - 1)
        add(sym, NR)
        add(full, NR - 1)
        s *= 2
    return fl, by, launches


def kernel_source_digest(text: str | None = None) -> str:
    """Digest of the block-product GEMM's source: the k_gemm kernel and its
    launch code in k_dense.hip (from its header comment to the explicit
    instantiations of plan_gemm), common.h, and from group.h the workgroup
    mapping (group_item, xcd_linear) and the GemmItem descriptor it reads."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2211_07572_amd", "csrc")
    if text is None:
        text = open(os.path.join(csrc, "k_dense.hip")).read()
    a = text.index("// Tiled MFMA GEMM")
    b = text.index("template void plan_gemm<double>")
    h = hashlib.sha256(text[a:b].encode())
    h.update(open(os.path.join(csrc, "common.h"), "rb").read())
    grp = open(os.path.join(csrc, "group.h")).read()
    for start, end in (("// Item owning workgroup bx", "// Refinement passes issued"),
                       ("// One product C = beta C", "// One block-vector product")):
        h.update(grp[grp.index(start):grp.index(end)].encode())
    return h.hexdigest()[:16]


def measured_traffic(name: str):
    """HBM bytes per launch from a committed counter summary, or None when the
    kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != kernel_source_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters: 3 copies of 2 GiB (float64)."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8,
                      "copies": 3}))


def run_gpu(w: G.Workload, precision: int, steps: int, warmup: int, kappa, f, odd_even: bool,
            shift=None):
    """W untimed steps, then K timed ones.  Returns the mean time per step over
    the K steps (one interval, synchronized on both sides), the per-step times
    (each synchronized), the last solution, and per-step solve infos and phase
    times.  shift: optional device diagonal term (Helmholtz)."""
    import torch
    from paper_2211_07572_amd import slab as S
    torch.cuda.synchronize()
    infos = []
    phases = []

    def one():
        h = S.slab_factor(kappa, w.n2, w.n1, w.b, w.h, precision=precision, tol=1e-10, max_iter=10,
                          odd_even=odd_even, shift=shift)
        u = S.slab_solve(h, f)
        infos.append((h.last_info.iterations, h.last_info.max_relres))
        phases.append(h.phase_us())
        h.free()
        return u

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    infos.clear()
    phases.clear()
    per_step = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        u = one()   # every call returns after its work has finished
        per_step.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, per_step, u, infos, phases


def host_cpu() -> dict:
    """CPU model, logical CPUs and cores of the host (lscpu, else /proc/cpuinfo)."""
    info = {"model": "unknown", "logical_cpus": os.cpu_count()}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "Model name":
                info["model"] = v
            elif k == "Socket(s)":
                info["sockets"] = int(v)
            elif k == "Core(s) per socket":
                info["cores_per_socket"] = int(v)
            elif k == "Thread(s) per core":
                info["threads_per_core"] = int(v)
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    if info["model"] == "unknown":
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    info["model"] = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return info


def host_relres(w: G.Workload, kappa_np, f_np, u) -> float:
    """Max-over-columns relative residual of a GPU solution, recomputed on the
    host by the FP64 oracle's A (Sec. 5.1 relerr_res)."""
    from oracle import slab_oracle as O
    prob = O.make_problem(kappa_np, w.n2, w.n1, w.b, w.h)
    return float(O.relres(prob, u.cpu().numpy(), f_np).max())


def cpu_baseline(w: G.Workload, kappa_np: np.ndarray, f_np: np.ndarray, slabs: int = 1) -> dict:
    """The FP64 oracle timed on a bounded sample of the same workload and scaled.

    Sample: stage one for `slabs` slab(s) (banded LU + all 2n boundary solves),
    one step of Alg. 1 on n x n blocks, and the solve work of one slab and one
    Alg. 2 block step for the 16 right-hand sides; the estimate for the whole
    job is m times each per-slab / per-block figure.
    """
    import scipy.linalg as sla
    from oracle import slab_oracle as O
    t_setup = time.perf_counter()
    prob = O.make_problem(kappa_np, w.n2, w.n1, w.b, w.h)
    setup_s = time.perf_counter() - t_setup
    m, n = prob.m, prob.n2
    # stage one: slabs 1..slabs (each touches two interfaces)
    t0 = time.perf_counter()
    contrib = [O.slab_contributions(prob, s) for s in range(1, 1 + slabs)]
    t_slab = (time.perf_counter() - t0) / slabs
    C = contrib[0]
    Tjj = prob.block(prob.I_o(0), prob.I_o(0)).toarray() - C[(0, 0)]
    Tup = -C[(0, 1)]
    Tlo = -C[(1, 0)]
    T11 = prob.block(prob.I_o(1), prob.I_o(1)).toarray() - C[(1, 1)]
    # one step of Alg. 1: factor S_j, form S_{j+1}
    t0 = time.perf_counter()
    lu = sla.lu_factor(Tjj)
    S1 = T11 - Tlo @ sla.lu_solve(lu, Tup)
    sla.lu_factor(S1)
    t_step = time.perf_counter() - t0
    # solve: one slab's reduced RHS and interior solve, one Alg. 2 block step
    fac1 = O.SlabFactor(prob.block(prob.I_e(1), prob.I_e(1)), w.b)
    F = f_np.reshape(f_np.shape[0], -1)
    t0 = time.perf_counter()
    y = fac1.solve(F[:, prob.I_e(1)].T)
    _ = prob.block(prob.I_o(1), prob.I_e(1)) @ y
    _ = fac1.solve(F[:, prob.I_e(1)].T)
    t_solve_slab = time.perf_counter() - t0
    g = F[:, prob.I_o(1)].T.copy()
    t0 = time.perf_counter()
    g -= Tlo @ sla.lu_solve(lu, g)
    g = sla.lu_solve(lu, g)
    g -= sla.lu_solve(lu, Tup @ g)
    t_solve_blk = time.perf_counter() - t0
    total = m * t_slab + (m - 1) * t_step + m * t_solve_slab + m * t_solve_blk
    sampled = slabs * t_slab + t_step + t_solve_slab + t_solve_blk
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": w.N / total, "unit": "DOF/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle (NumPy/SciPy-LAPACK, {threads} BLAS threads) timed on "
                       f"{slabs} slab of stage one, 1 step of Alg. 1, 1 slab + 1 block of the "
                       f"16-RHS solve ({sampled:.1f} s), scaled by m={m}: an ESTIMATE of "
                       f"{total:.0f} s for the whole job, not a measurement of it"),
            "estimated_total_s": total, "sampled_s": sampled, "setup_s": setup_s,
            "host_cpu": host_cpu()}


def cpu_oracle_whole(w: G.Workload, workers: int, one_core: bool = False) -> dict:
    """The whole job of workload w (factor + 1-RHS solve) on the FP64 oracle,
    measured: stage one with its independent slabs spread over a process pool
    of `workers` processes (one BLAS thread each), stage two (Alg. 1, LAPACK)
    and the solve (Alg. 4) in this process; one_core: everything on one
    thread (one BLAS thread, no pool)."""
    from oracle import slab_oracle as O
    prob = O.make_problem(w.kappa(), w.n2, w.n1, w.b, w.h)
    f = w.rhs(1)

    def run():
        t0 = time.perf_counter()
        fac = O.factor(prob, workers=workers)
        t1 = time.perf_counter()
        u = O.solve(fac, f)
        t2 = time.perf_counter()
        return t0, t1, t2, u
    if one_core:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            t0, t1, t2, u = run()
    else:
        t0, t1, t2, u = run()
    return {"value": w.N / (t2 - t0), "unit": "DOF/s", "kind": "oracle",
            "cores": 1 if one_core else workers,
            "sample": f"the whole {w.name} job, 1 RHS, measured (not extrapolated)",
            "factor_s": t1 - t0, "solve_s": t2 - t1,
            "relres": float(O.relres(prob, u, f).max())}


def extra_workloads(warmup: int, steps: int) -> dict:
    """The 1024x1024 (FP64, 1 and 64 right-hand sides; mixed, 1 RHS) and
    512x512 (FP64 factor + solve + adjoint + gradient) workloads, the
    indefinite Helmholtz workloads (40 points per wavelength, and the paper's
    J0 benchmark at 1M and 4M unknowns) on the GPU, median step times."""
    import torch
    from paper_2211_07572_amd import slab as S
    out = {}
    w = G.DIFFUSION_1024
    kap = torch.as_tensor(w.kappa(), device="cuda")
    for nrhs in (1, 64):
        f = torch.as_tensor(w.rhs(nrhs), device="cuda").contiguous()
        for name, prec in (("fp64", S.SLAB_FP64), ("mixed", S.SLAB_MIXED)):
            if name == "mixed" and nrhs == 64:
                continue
            _, per, _, info, _ = run_gpu(w, prec, steps, warmup, kap, f, True)
            med = float(np.median(per))
            out[f"{w.name}_{name}_nrhs{nrhs}"] = {
                "ms_per_step": med * 1e3, "dof_per_s": w.N / med, "nrhs": nrhs,
                "max_relres": max(r for _, r in info), "refine_passes": max(i for i, _ in info)}
    out[f"{G.ADJOINT_512.name}_batch16_fp64_factor_solve_adjoint_grad"] = differentiation_batch(
        warmup, steps)
    out.update(helmholtz_workload(warmup, steps))
    out.update(helmholtz_fd_paper(warmup, steps))
    return out


# The paper's FD Helmholtz runs at 250 points per wavelength (Sec. 5.2, the
# figure of constant points-per-wavelength runs): N, b, kappa, the memory M of
# the factorization, relerr_res, relerr_true and T_solve (one RHS, on its CPU)
# of its first two rows.
PAPER_FD_ROWS = [
    {"N": 1.0e6, "b": 50, "kappa": 27.1, "M_GB": 0.5, "relerr_res": 1.1e-11,
     "relerr_true": 1.8e-3, "T_solve_s": 0.9},
    {"N": 4.0e6, "b": 100, "kappa": 52.3, "M_GB": 2.5, "relerr_res": 1.8e-11,
     "relerr_true": 2.6e-3, "T_solve_s": 2.9},
]


def helmholtz_fd_paper(warmup: int, steps: int) -> dict:
    """The paper's FD Helmholtz benchmark (-Laplace u - kappa^2 u = 0 on the
    unit square, Dirichlet data from u_true = J0(kappa |x - (-0.1, 0.5)|)) at
    its first two sizes: n = 1000 and 2000 per side (h = 1/(n+1)), b = 49 (the
    largest width whose period divides n; the paper's b is 50 and 100), FP64,
    odd-even order.  One step: factor, load of the boundary data, solve.
    relerr_res and relerr_true are reported beside the paper's printed ones
    (its T_solve is on its CPU: context only)."""
    import torch
    from paper_2211_07572_amd import slab as S
    out = {}
    log("extra workload: the paper's FD Helmholtz benchmark (J0 data), 1M and 4M unknowns")
    for row in PAPER_FD_ROWS:
        n = int(round(np.sqrt(row["N"])))
        k = row["kappa"]
        h = 1.0 / (n + 1)
        ut = G.bessel_field(n, n, k, h)
        kap = torch.as_tensor(G.kappa_const(n, n), device="cuda")
        cd = torch.full((n, n), -k * k, dtype=torch.float64, device="cuda")
        g = torch.as_tensor(ut, device="cuda")
        times, solve_times = [], []
        for it in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hd = S.slab_factor(kap, n, n, 49, h, odd_even=True, shift=cd)
            f = S.slab_dirichlet_load(hd, g)
            t1 = time.perf_counter()
            u = S.slab_solve(hd, f)   # returns after its work has finished
            t2 = time.perf_counter()
            if it >= warmup:
                times.append(t2 - t0)
                solve_times.append(t2 - t1)
            if it < warmup + steps - 1:
                hd.free()
        rr = S.slab_residual(hd, f, u)[0]
        passes = hd.last_info.iterations
        neg = hd.negative_pivots()
        held = hd.query(5)   # device bytes the factored handle keeps (the paper's M)
        hd.free()
        e = float(np.linalg.norm(u.cpu().numpy()[0] - ut[1:-1, 1:-1]) /
                  np.linalg.norm(ut[1:-1, 1:-1]))
        med = float(np.median(times))
        out[f"helmholtz_fd_j0_{n}x{n}_b49_kappa{k}_fp64"] = {
            "ms_per_step": med * 1e3, "dof_per_s": n * n / med,
            "solve_ms": float(np.median(solve_times)) * 1e3, "relerr_res": rr,
            "relerr_true": e, "refine_passes": passes, "negative_pivots": neg,
            "memory_GB": held / 1e9, "paper": row, "steps": steps, "warmup": warmup}
    return out


def helmholtz_workload(warmup: int, steps: int) -> dict:
    """Indefinite Helmholtz, -Laplace u - k^2 u, factor + solve per step in FP64
    (odd-even order, signed elimination): 1024 x 1024, b = 15, 40 points per
    wavelength (definite slabs, indefinite T) and 2048 x 2048, b = 31, 20 points
    per wavelength (indefinite slabs too).  The negative pivots of T are
    reported beside their closed-form count (the sine modes: eigenvalues of A
    below k^2 less m times those of one slab interior), with cond(A) from the
    same eigenvalues, and the outcome of the mixed form (one untimed solve)."""
    import torch
    from paper_2211_07572_amd import slab as S
    log("extra workload: indefinite Helmholtz 1024x1024 (40 points per wavelength) and "
        "2048x2048 (20)")

    def laplace_eigs(n2, n1, h):
        p1 = np.arange(1, n1 + 1)[:, None]
        p2 = np.arange(1, n2 + 1)[None, :]
        return (4 - 2 * np.cos(np.pi * p1 / (n1 + 1)) - 2 * np.cos(np.pi * p2 / (n2 + 1))) / h ** 2

    out = {}
    for w in (G.HELMHOLTZ_1024, G.HELMHOLTZ_2048):
        c = w.shift()
        k2 = -float(c[0, 0])
        lam = laplace_eigs(w.n2, w.n1, w.h)
        gap = np.abs(lam - k2)
        neg_closed = int((lam < k2).sum()) - w.m * int((laplace_eigs(w.n2, w.b, w.h) < k2).sum())
        kap = torch.as_tensor(w.kappa(), device="cuda")
        cd = torch.as_tensor(c, device="cuda")
        f = torch.as_tensor(w.rhs(1), device="cuda").contiguous()
        _, per, _, info, _ = run_gpu(w, S.SLAB_FP64, steps, warmup, kap, f, True, shift=cd)
        h = S.slab_factor(kap, w.n2, w.n1, w.b, w.h, precision=S.SLAB_FP64, odd_even=True,
                          shift=cd)
        neg = h.negative_pivots()
        h.free()
        med = float(np.median(per))
        res = {"ms_per_step": med * 1e3, "dof_per_s": w.N / med,
               "max_relres": max(r for _, r in info), "refine_passes": max(i for i, _ in info),
               "negative_pivots": neg, "negative_pivots_closed_form": neg_closed,
               "cond_A": float(gap.max() / gap.min()), "steps": steps, "warmup": warmup}
        # the FP32 reduced factorization (mixed form) converges only while cond(T)
        # times its growth times the FP32 rounding stays below one: its outcome
        # here (one untimed solve, not checked)
        h = S.slab_factor(kap, w.n2, w.n1, w.b, w.h, precision=S.SLAB_MIXED, odd_even=True,
                          shift=cd, max_iter=10)
        S.slab_solve(h, f, check=False)
        rr = h.last_info.max_relres
        res["mixed_form"] = {"refine_passes": h.last_info.iterations,
                             "max_relres": rr if np.isfinite(rr) else None,
                             "converged": bool(rr <= 1e-10)}
        h.free()
        out[f"{w.name}_fp64"] = res
    return out


def sketch_workload(w: G.Workload, kappa, warmup: int, steps: int) -> dict:
    """Matrix-free products with the reduced matrix, Y = T Omega, for s = 6b
    Gaussian test vectors on grid w (mixed precision: FP64 slab sweeps), the
    product the paper's randomized sketches of T are formed from.  One step is
    one slab_apply_reduced call on a factored handle (factorization untimed)."""
    import torch
    from paper_2211_07572_amd import slab as S
    s = 6 * w.b
    h = S.slab_factor(kappa, w.n2, w.n1, w.b, w.h, precision=S.SLAB_MIXED, odd_even=True)
    x = torch.as_tensor(G.gaussian_test_vectors(w.m, s, w.n2), device="cuda")
    times = []
    for it in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.slab_apply_reduced(h, x)      # synchronizes at its end
        if it >= warmup:
            times.append(time.perf_counter() - t0)
    h.free()
    med = float(np.median(times))
    return {"ms_per_step": med * 1e3, "test_vectors": s, "vectors_per_s": s / med,
            "slab_factor_reads_GBps": 2.0 * w.m * w.n2 * 32 * 32 * 8 / med / 1e9,
            "steps": steps, "warmup": warmup}


def differentiation_batch(warmup: int, steps: int) -> dict:
    """The 512x512 differentiation workload (b = 15): 16 fields theta_i = log
    kappa_i factored together (FP64, odd-even order), the shared load solved,
    the adjoint of L_i = 1/2 ||u_i - u_obs||^2 solved and dL/dtheta_i formed,
    all as batches.  u_obs is a stand-in here (the load itself): the cost of a
    step does not depend on it."""
    import torch
    from paper_2211_07572_amd import slab as S
    w = G.ADJOINT_512
    thetas = [torch.as_tensor(G.grf(w.n2, w.n1, s, w.h), device="cuda")
              for s in G.DIFF_THETA_SEEDS]
    B = len(thetas)
    f = torch.as_tensor(w.rhs(1), device="cuda").contiguous()
    times = []
    for it in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt = S.slab_factor_batch(thetas, [(w.n2, w.n1, w.b, w.h)] * B, precision=S.SLAB_FP64,
                                 coef_log=True)
        us = S.slab_solve_batch(bt, [f] * B)
        lams = S.slab_solve_adjoint_batch(bt, [u - f for u in us])
        S.slab_kappa_grad_batch(bt, us, lams, mode=1)
        torch.cuda.synchronize()
        if it >= warmup:
            times.append(time.perf_counter() - t0)
        bt.free()
    med = float(np.median(times))
    return {"ms_per_step": med * 1e3, "fields": B, "dof_per_s": B * w.N / med,
            "steps": steps, "warmup": warmup}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    from paper_2211_07572_amd import slab as S
    S.load_library()
    if args.workload == "batch256":
        print(json.dumps(finite_json(run_batch_line(args)), allow_nan=False))
        return
    w = workload(args.workload)
    kappa_np = w.kappa()
    f_np = w.rhs()
    kappa = torch.as_tensor(kappa_np, device="cuda")
    f = torch.as_tensor(f_np, device="cuda").contiguous()
    torch.cuda.synchronize()

    prec = {"mixed": S.SLAB_MIXED, "fp32": S.SLAB_FP32_REFINE}[args.precision]
    oe = args.order == "odd_even"
    log(f"headline: {w.name}, {args.precision}, {args.order}")
    dt32, per32, u32, info32, ph32 = run_gpu(w, prec, args.steps, args.warmup, kappa, f, oe)
    relres32 = max(r for _, r in info32)
    iters32 = max(i for i, _ in info32)
    ph = {k: float(np.median([p[k] for p in ph32])) for k in ph32[0]}
    result = {
        "metric": "factor+solve DOF/s, FP32+refine vs FP64 on GPU at rel. residual 1e-10",
        "value": w.N / dt32,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n2": w.n2, "n1": w.n1, "b": w.b, "slabs": w.m,
                   "nrhs": w.nrhs, "N": w.N, "kappa": "exp(GRF l=0.05 var=1)",
                   "rhs": "N(0,1)", "tol": 1e-10,
                   "precision": {"mixed": "FP64 slab work, FP32 reduced system, FP64 refinement",
                                 "fp32": "FP32 throughout, FP64 sum forming T, FP64 refinement"}[args.precision],
                   "stage_two": {"odd_even": "odd-even elimination order",
                                 "sweep": "sweep of Alg. 1"}[args.order]},
        "max_relres": relres32,
        "max_relres_host": host_relres(w, kappa_np, f_np, u32),
        "step_ms": [t * 1e3 for t in per32],
        "refine_passes": iters32,
        "phase_ms": {k: v / 1e3 for k, v in ph.items()},
    }
    # roofline of the dominant kernel: the block products of stage two (k_gemm,
    # FP32 MFMA), timed by HIP events recorded on the factor's stream around
    # each of its launches (summed); achieved = algorithmic flops / time
    fl_bp, by_bp, n_bp = block_products(w, oe)
    t_bp = ph["block_products"] / 1e6
    traffic = measured_traffic("traffic_k_gemm_block_products_2048x4096_b31.md")
    result["roofline"] = {"kernel": "k_gemm<float> (block products of stage two)",
                          "bound": "mfma", "achieved": fl_bp / t_bp / 1e12,
                          "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                          "frac": fl_bp / t_bp / 1e12 / PEAK_TFLOPS["f32"],
                          "traffic": traffic,
                          "algorithmic_bytes_per_launch": by_bp / n_bp,
                          "flops_per_launch": fl_bp / n_bp, "launches": n_bp,
                          "avg_launch_ms": t_bp / n_bp * 1e3}
    # the Schur propagation (one launch per factor) beside it
    t_schur = ph["schur"] / 1e6
    fl = schur_flops(w)
    dt = "f64" if args.precision == "mixed" else "f32"
    result["roofline_schur"] = {"kernel": f"k_schur<{'double' if dt == 'f64' else 'float'},32>",
                                "bound": "mfma", "achieved": fl / t_schur / 1e12,
                                "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                                "frac": fl / t_schur / 1e12 / PEAK_TFLOPS[dt]}
    tb = ph["block_factor"] / 1e6
    result["block_factor_tflops"] = block_factor_flops(w, oe) / tb / 1e12

    # the compared forms run with the same warm-up and step counts as the
    # headline (at least 1 and 3); ms_per_step is the median step
    cw, cs = max(args.warmup, 1), max(args.steps, 3)

    def form(precision, odd_even):
        dto, per_o, _, info_o, ph_o = run_gpu(w, precision, cs, cw, kappa, f, odd_even)
        pm = {k: float(np.median([p[k] for p in ph_o])) / 1e3 for k in ph_o[0]}
        med = float(np.median(per_o))
        return med, {"value": w.N / med, "ms_per_step": med * 1e3, "mean_ms": dto * 1e3,
                     "steps": cs, "warmup": cw,
                     "max_relres": max(r for _, r in info_o),
                     "refine_passes": max(i for i, _ in info_o), "phase_ms": pm,
                     "block_factor_tflops": block_factor_flops(w, odd_even) / (pm["block_factor"] / 1e3) / 1e12}
    if not args.skip_other:
        other = "fp32" if args.precision == "mixed" else "mixed"
        log(f"{other} form")
        result[f"{other}_form"] = form({"mixed": S.SLAB_MIXED, "fp32": S.SLAB_FP32_REFINE}[other], oe)[1]
        other_order = "sweep" if oe else "odd_even"
        log(f"{other_order} order")
        result[f"{other_order}_order"] = form(prec, not oe)[1]
    if args.autotune:
        # slab width picked by the autotuner for this grid (the configuration fixes b)
        t0 = time.perf_counter()
        bt, times = S.slab_autotune(kappa, w.n2, w.n1, w.h, precision=prec, odd_even=oe,
                                    nrhs=w.nrhs)
        result["autotune"] = {"b": bt, "seconds_per_candidate": {str(k): v for k, v in times.items()},
                              "tuning_s": time.perf_counter() - t0}
    if not args.skip_fp64:
        log("fp64 form")
        dt64, res64 = form(S.SLAB_FP64, oe)
        result["fp64"] = res64
        result["fp32_refine_speedup_vs_fp64"] = dt64 / float(np.median(per32))
    if not args.skip_extra:
        log("extra workloads: 1024x1024, 512x512 batch of 16")
        result["extra_workloads"] = extra_workloads(cw, cs)
        log("extra workload: sketch of T")
        result["extra_workloads"][f"{w.name}_sketch_T_6b"] = sketch_workload(w, kappa, cw, cs)
        log("extra workload: batch of 256")
        result["extra_workloads"]["batch256_uneven"] = run_batch(cw, cs)
    if not args.skip_cpu:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(w, kappa_np, f_np, args.cpu_slabs)
        workers = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log("oracle: whole 64x64 job (1 core, all cores) and whole 1024x1024 job")
        result["cpu_oracle_whole_jobs"] = {
            "host_cpu": host_cpu(),
            "poisson_64x64_b7_1core": cpu_oracle_whole(G.POISSON_64, 1, one_core=True),
            f"poisson_64x64_b7_{workers}workers": cpu_oracle_whole(G.POISSON_64, workers),
            f"diffusion_1024x1024_b31_{workers}workers": cpu_oracle_whole(G.DIFFUSION_1024, workers),
        }
    print(json.dumps(finite_json(result), allow_nan=False))


if __name__ == "__main__":
    main()
