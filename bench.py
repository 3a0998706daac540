"""Benchmark: FD-preconditioned space-time PCG on one MI355X.

One step = the right-hand side with lifting (lifting solve on the faces,
then f_bar = (f - S_V u_bar, S_V B_I) by sum factorisation) followed by one
complete preconditioned CG solve of A u = f_bar to a relative residual of 1e-8
from a zero initial guess (matvec, FD preconditioner apply and PCG updates
every iteration); the sampled initial datum is already resident in HBM.
Workload: 2D space (unit square) + time, p = 3, 64^3 elements
(n_t = 66, n_s = 65 per direction, N = 278,850 free complex dofs), potential
V = sum of 8 seeded Gaussians (the preconditioner keeps V = 0), initial datum
a seeded wave packet (|k| <= 20), f = 0, homogeneous Dirichlet data.

Printed JSON line: value = N / (seconds per solve) / 1e6 [Mdof/s], plus the
preconditioner-apply throughput per precision, the time to 1e-8 per
preconditioner precision, the roofline of the dominant kernel (live HIP-event
timing) and the CPU oracle timed on a bounded sample.
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

METRIC = "FD precond apply Mdof/s + PCG time to 1e-8: FP64 vs mixed/batched/warm-start"
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector and matrix peak
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of the 2D p=3 matvec kernel on this workload: FETCH_SIZE and WRITE_SIZE passes
# of rocprofv3 over `bench.py --profile`, each scaled by what the same counter reads for a 64 MiB
# device copy in that run (x 1.999 and x 1.000); profiles/pcg_2d_p3_n64_gauss_traffic.md.  Valid for
# the matvec kernel as profiled (12.57 MB read + 4.47 MB written per launch, 705 blocks of 6 points).
MATVEC_KERNEL = "matvec_kernel<2,3,3,1>"
MATVEC_TRAFFIC_BYTES = 17.04e6


def build_workload(sample=0, n_el=64, p=3):
    from paper_2311_18461_amd import inputs, stfd
    w = inputs.gaussian_potential_2d_workload(sample, n_el=n_el, p=p)
    kt, ks = w.knots_t(), [w.knots_s()] * 2
    Vq = stfd.sample_on_quad_grid(w.potential, ks, p)
    prob = stfd.Problem(kt, ks, p, p, w.T, w.nu, V_quad=Vq, max_nrhs=1)
    return w, prob


def time_events(fn, reps, stream):
    import torch
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps  # ms


def batched_section(dev, stream, reps=3):
    """64 wave-packet systems (V = 0, p = 3) dealt over the grids 16^3 .. 64^3: one batched call
    (graph per iteration, one stream per grid) vs the same systems solved grid by grid and one by one."""
    import torch
    from paper_2311_18461_amd import inputs, stfd
    work = inputs.batched_2d_workload()
    probs, fs, us, nr = [], [], [], []
    for n_el, packets in work.items():
        kt, ks = inputs.uniform_open_knots(n_el, 3), [inputs.uniform_open_knots(n_el, 3)] * 2
        pr = stfd.Problem(kt, ks, 3, 3, 1.0, 1.0, max_nrhs=len(packets))
        u0 = torch.from_numpy(np.concatenate([pr.sample_space(w) for w in packets])).to(dev)
        f = torch.empty(pr.N * len(packets), dtype=torch.complex128, device=dev)
        pr.load_vector(f, u0_q=u0, nrhs=len(packets), stream=stream)
        probs.append(pr)
        fs.append(f)
        us.append(torch.empty_like(f))
        nr.append(len(packets))
    total = sum(pr.N * n for pr, n in zip(probs, nr))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3, out

    t_batch, (rc, info) = timed(lambda: stfd.pcg_solve_batched(probs, fs, us, nr, rtol=1e-8, maxit=1000,
                                                                stream=stream))
    t_grid, _ = timed(lambda: [pr.pcg_solve(f, u, nrhs=n, rtol=1e-8, maxit=1000, stream=stream)
                               for pr, f, u, n in zip(probs, fs, us, nr)])

    def one_by_one():
        for pr, f, u, n in zip(probs, fs, us, nr):
            for j in range(n):
                pr.pcg_solve(f[j * pr.N:(j + 1) * pr.N], u[j * pr.N:(j + 1) * pr.N], rtol=1e-8, maxit=1000,
                             stream=stream)
    t_one, _ = timed(one_by_one)
    its = [i["iters"] for i in info]
    return {"systems": len(its), "grids": list(work.keys()), "systems_per_grid": nr, "total_dofs": total,
            "batched_ms": round(t_batch, 3), "batched_mdofs": round(total / (t_batch * 1e-3) / 1e6, 2),
            "grid_by_grid_ms": round(t_grid, 3), "one_by_one_ms": round(t_one, 3),
            "iterations_min_max": [min(its), max(its)],
            "max_true_rel_res": float(f"{max(i['true_rel_res'] for i in info):.3e}")}


WARMSTART_WEIGHTS = os.path.join(ROOT, "paper_2311_18461_amd", "data", "warmstart_annulus_p4_n64.npz")


def warmstart_section(stream, n_eval=20):
    """Learned warm start on the quarter-annulus workload (p = 4, 64^3): cold vs warm PCG on the
    first n_eval held-out seeds with the trained network (training: warmstart.py train)."""
    from paper_2311_18461_amd import warmstart
    if not os.path.exists(WARMSTART_WEIGHTS):
        return {"skipped": "no trained weights in paper_2311_18461_amd/data"}
    wl = warmstart.AnnulusWorkload(stream=stream)
    net = warmstart.load_net(wl, WARMSTART_WEIGHTS)
    rows = warmstart.evaluate(wl, net, warmstart.TEST_SEED0, n_eval)
    out = warmstart.summarize(rows)
    out["held_out_seeds"] = [warmstart.TEST_SEED0, warmstart.TEST_SEED0 + n_eval - 1]
    out["n_dof_free"] = wl.N
    return out


def precision_3d_section(stream, cases=((48, 3), (32, 4)), bf16_maxit=300):
    """3D space + time with the seeded harmonic potential (p = 3 at 48^4 elements, p = 4 at 32^4):
    FD apply throughput and error of the FP32 and BF16 mode products against the FP64 apply on the
    same input, and PCG to 1e-8 per preconditioner precision (FP64 outer loop; BF16 capped)."""
    import torch
    from paper_2311_18461_amd import inputs, stfd
    dev = torch.device("cuda:0")
    out = {}
    for n_el, p in cases:
        w = inputs.harmonic_3d_workload(0, n_el=n_el, p=p, with_potential=True)
        ks = [w.knots_s()] * 3
        t0 = time.perf_counter()
        prob = stfd.Problem(w.knots_t(), ks, p, p, w.T, w.nu, V_quad=stfd.sample_on_quad_grid(w.potential, ks, p))
        torch.cuda.synchronize()
        row = {"n_dof_free": prob.N, "setup_s": round(time.perf_counter() - t0, 2)}
        r = torch.from_numpy(inputs.random_complex(prob.N, 3999)).to(dev)
        z = torch.empty_like(r)
        z64 = torch.empty_like(r)
        for prec in ("fp64", "fp32", "bf16"):
            prob.apply_preconditioner(r, z, precision=prec, stream=stream)
            ms = time_events(lambda: prob.apply_preconditioner(r, z, precision=prec, stream=stream), 10, stream)
            if prec == "fp64":
                z64.copy_(z)
            err = float(torch.linalg.vector_norm(z - z64) / torch.linalg.vector_norm(z64))
            row[prec] = {"apply_ms": round(ms, 4), "apply_mdofs": round(prob.N / (ms * 1e-3) / 1e6, 1),
                         "apply_relerr_vs_fp64": float(f"{err:.3e}")}
        row["matvec_ms"] = round(time_events(lambda: prob.matvec(r, z, stream=stream), 10, stream), 4)
        f = torch.empty_like(r)
        prob.load_vector(f, u0_q=torch.from_numpy(prob.sample_space(w.u0)).to(dev), stream=stream)
        u = torch.empty_like(r)
        for prec in ("fp64", "fp32", "bf16"):
            maxit = bf16_maxit if prec == "bf16" else 1000
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rc, info = prob.pcg_solve(f, u, rtol=1e-8, maxit=maxit, precision=prec, stream=stream)
            torch.cuda.synchronize()
            row[prec].update({"pcg_ms": round((time.perf_counter() - t1) * 1e3, 2), "pcg_iterations": info[0]["iters"],
                              "pcg_converged": rc == stfd.OK, "pcg_true_rel_res": float(f"{info[0]['true_rel_res']:.3e}")})
        prob.close()
        out[f"p{p}_n{n_el}_harmonic"] = row
    return out


def cpu_baseline(w, budget_s=20.0):
    """The oracle (FP64 NumPy/SciPy, all host cores): right-hand side with lifting, then PCG to 1e-8,
    on the same workload (setup excluded)."""
    from threadpoolctl import threadpool_info
    from oracle.operators import FastDiagonalization, Problem as OProblem
    from oracle.pcg import pcg
    from oracle.rhs import SpaceTimeBasis, assemble_rhs
    ks = [w.knots_s()] * 2
    ref = OProblem(w.knots_t(), ks, w.p, w.p, w.nu, w.potential)
    fd = FastDiagonalization(ref)
    stb = SpaceTimeBasis(w.knots_t(), ks, w.p, w.p)
    times, t_rhs, iters = [], [], []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        fb, _ = assemble_rhs(stb, w.nu, u0=w.u0, V=w.potential)
        t1 = time.perf_counter()
        _, info = pcg(ref.matvec, fd.apply, fb, tol=1e-8, maxit=1000)
        times.append(time.perf_counter() - t0)
        t_rhs.append(t1 - t0)
        iters.append(info["iters"])
        if time.perf_counter() - t_start > budget_s * 0.5 or len(times) >= 5:
            break
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    t = float(np.median(times))
    return {"value": ref.N / t / 1e6, "unit": "Mdof/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(times)} complete steps of the same workload (right-hand side with lifting "
                      f"{np.median(t_rhs):.2f} s + FP64 PCG to 1e-8, {iters[0]} iterations), median {t:.3f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D precision section")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: one solve, 20 applies and matvecs, and a device copy of "
                         "known size (64 MiB read + 64 MiB written) to calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2311_18461_amd import inputs, stfd
    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    w, prob = build_workload()
    N = prob.N
    u0_q = torch.from_numpy(prob.sample_space(w.u0)).to(dev)  # initial datum on the Gauss grid
    f = torch.empty(N, dtype=torch.complex128, device=dev)
    u = torch.empty_like(f)

    def rhs():
        prob.load_vector(f, u0_q=u0_q, stream=stream)

    def solve(prec=args.precision):
        return prob.pcg_solve(f, u, rtol=1e-8, maxit=1000, precision=prec, stream=stream)

    def step(prec=args.precision):
        rhs()
        return solve(prec)

    if args.profile:
        step()
        rc, info = step()
        r = torch.from_numpy(inputs.random_complex(N, 2998)).to(dev)
        s = torch.empty_like(r)
        for _ in range(20):
            prob.apply_preconditioner(r, s, stream=stream)
        for _ in range(20):
            prob.matvec(r, s, stream=stream)
        src = torch.ones(8 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "iterations": info[0]["iters"], "copy_bytes": src.numel() * 8}))
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    iters = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, info = step()
        iters.append(info[0]["iters"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    value = N / (ms_per_step / 1e3) / 1e6

    # right-hand side alone (lifting + load vector)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        rhs()
    torch.cuda.synchronize()
    rhs_ms = (time.perf_counter() - t1) / 5 * 1e3

    # time to 1e-8 per preconditioner precision (a few solves each)
    pcg_ms, pcg_iters, pcg_true = {}, {}, {}
    for prec in ("fp64", "fp32", "bf16"):
        solve(prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            rc, info = solve(prec)
        torch.cuda.synchronize()
        pcg_ms[prec] = (time.perf_counter() - t1) / 5 * 1e3
        pcg_iters[prec] = info[0]["iters"]
        pcg_true[prec] = info[0]["true_rel_res"]

    # the same solve with every iteration replayed from a captured graph
    prob.pcg_solve(f, u, rtol=1e-8, maxit=1000, stream=stream, graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        rc, info = prob.pcg_solve(f, u, rtol=1e-8, maxit=1000, stream=stream, graph=True)
    torch.cuda.synchronize()
    pcg_graph_ms = (time.perf_counter() - t1) / 5 * 1e3

    # apply and matvec throughput with HIP events on the launch stream
    r = torch.from_numpy(inputs.random_complex(N, 2998)).to(dev)
    s = torch.empty_like(r)
    apply_ms = {}
    for prec in ("fp64", "fp32", "bf16"):
        prob.apply_preconditioner(r, s, precision=prec, stream=stream)
        apply_ms[prec] = time_events(lambda: prob.apply_preconditioner(r, s, precision=prec, stream=stream), 50,
                                     stream)
    prob.matvec(r, s, stream=stream)
    matvec_ms = time_events(lambda: prob.matvec(r, s, stream=stream), 50, stream)

    # dominant kernel: the system matvec (one launch per call); algorithmic FP64 work per dof:
    # 3 real (2p+1)^d-point stencils on complex data + 3 complex-by-real (2p+1)-band time products
    p, d = w.p, 2
    flops_per_dof = 12 * ((2 * p + 1) ** d + 2 * p + 1)
    achieved = flops_per_dof * N / (matvec_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": MATVEC_KERNEL, "achieved": round(achieved, 3),
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": MATVEC_TRAFFIC_BYTES, "traffic_unit": "bytes per launch (rocprofv3 FETCH/WRITE_SIZE, "
                                                               "copy-calibrated)",
                "traffic_algorithmic": 16 * 2 * N + 24 * 49 * prob.N_s,
                "traffic_gbs": round(MATVEC_TRAFFIC_BYTES / (matvec_ms * 1e-3) / 1e9, 1),
                "avg_launch_us": round(matvec_ms * 1e3, 2), "flops_per_dof": flops_per_dof}

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mdof/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else f"f64+{args.precision}",
        "data": "synthetic",
        "config": {"workload": "2D space + time, p=3, 64^3 elements, 8-Gaussian potential (seed 2000), "
                               "wave-packet initial datum (seed 2500), f = 0; right-hand side with lifting + "
                               "PCG to 1e-8 from x0=0",
                   "n_dof_free": N, "n_t": prob.n_t, "n_s": prob.n_s,
                   "preconditioner_precision": args.precision},
        "iterations": int(np.median(iters)),
        "rhs_ms": round(rhs_ms, 4),
        "pcg_ms_to_1e-8": {k: round(v, 4) for k, v in pcg_ms.items()},
        "pcg_iterations": pcg_iters,
        "pcg_true_rel_res": {k: float(f"{v:.3e}") for k, v in pcg_true.items()},
        "pcg_graph_ms_to_1e-8": round(pcg_graph_ms, 4),
        "fd_apply_mdofs": {k: round(N / (v * 1e-3) / 1e6, 1) for k, v in apply_ms.items()},
        "fd_apply_us": {k: round(v * 1e3, 2) for k, v in apply_ms.items()},
        "matvec_us": round(matvec_ms * 1e3, 2),
        "roofline": roofline,
    }
    out["batched"] = batched_section(dev, stream)
    out["warm_start"] = warmstart_section(stream)
    if not args.no_3d:
        out["precision_3d"] = precision_3d_section(stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
