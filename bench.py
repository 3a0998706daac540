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
import gc
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
# Dominant kernel of the step: the FP64 mode product of the FD apply (Algorithm 1 steps 2 and 4;
# rocprofv3 kernel statistics of `bench.py --profile 2d`: 24.4% of kernel time, plus 9.8% for its
# variant with the fused PCG dot products).  Per launch on this workload (2D p=3 64^3, n = 65 per
# direction), from profiles/fd_apply_2d_p3_n64_gauss.md (mean of its two launch shapes):
#   HBM traffic: FETCH_SIZE x 1.999 + WRITE_SIZE x 1.000 (factors: what the counters read for a
#   64 MiB device copy in the same run) = 9.44e6 bytes (algorithmic: 32 bytes per dof = 8.92e6);
#   MFMA work: SQ_INSTS_VALU_MFMA_MOPS_F64 x 512 = 9.77e7 flops (algorithmic 4 n = 260 flops per
#   dof = 7.25e7; the rest is the padding of n = 65 to 68 rows of K and 80 output columns).
# The bench times the launch with HIP events on its stream around 500 back-to-back launches
# (stfd_time_mode_product: per launch, the kernel plus what its dispatch does not overlap with the
# previous one); the events around each single launch of an apply (library timing hooks) enclose the
# whole dispatch as well and are reported beside it.
MODE_PRODUCT_KERNEL = "mode_product_kernel<0, double, double, 17, 1, false, 0, true>"
MODE_PRODUCT_TRAFFIC_BYTES = 9.44e6
MODE_PRODUCT_MFMA_FLOPS = 9.77e7
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


def batched_section(dev, stream, reps=5):
    """64 wave-packet systems (V = 0, p = 3) dealt over the grids 16^3 .. 64^3: one batched call
    (one stream per grid; also with each grid's iteration replayed from a captured graph) vs the same
    systems solved grid by grid and one by one."""
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
        # median of individually synchronised calls after one untimed call (a host-side pause, such
        # as the garbage collector freeing an earlier section's buffers, then moves one sample only)
        gc.collect()
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ts)), out

    t_batch, (rc, info) = timed(lambda: stfd.pcg_solve_batched(probs, fs, us, nr, rtol=1e-8, maxit=1000,
                                                                stream=stream))
    t_batch_graph, _ = timed(lambda: stfd.pcg_solve_batched(probs, fs, us, nr, rtol=1e-8, maxit=1000,
                                                           stream=stream, graph=True))
    t_grid, _ = timed(lambda: [pr.pcg_solve(f, u, nrhs=n, rtol=1e-8, maxit=1000, stream=stream)
                               for pr, f, u, n in zip(probs, fs, us, nr)])

    def one_by_one():
        for pr, f, u, n in zip(probs, fs, us, nr):
            for j in range(n):
                pr.pcg_solve(f[j * pr.N:(j + 1) * pr.N], u[j * pr.N:(j + 1) * pr.N], rtol=1e-8, maxit=1000,
                             stream=stream)
    t_one, _ = timed(one_by_one)
    its = [i["iters"] for i in info]
    # one FD apply of all 64 systems: every grid's stacked apply on its own stream (default
    # priority), against the same applies one grid after the other, and the HBM roof of Algorithm
    # 1 steps 2-4 (96 bytes per dof: three passes of the complex FP64 tensor)
    rs = [torch.from_numpy(inputs.random_complex(pr.N * n, 77)).to(dev) for pr, n in zip(probs, nr)]
    zs = [torch.empty_like(r) for r in rs]
    side = [torch.cuda.Stream() for _ in probs]

    def apply_all(concurrent):
        if concurrent:
            ev = torch.cuda.Event()
            ev.record(stream)
            for pr, r, z, n, st in zip(probs, rs, zs, nr, side):
                st.wait_event(ev)
                pr.apply_preconditioner(r, z, nrhs=n, stream=st)
            for st in side:
                stream.wait_stream(st)
        else:
            for pr, r, z, n in zip(probs, rs, zs, nr):
                pr.apply_preconditioner(r, z, nrhs=n, stream=stream)

    apply_all(True)
    apply_all(False)
    ms_conc = time_events(lambda: apply_all(True), 20, stream)
    ms_seq = time_events(lambda: apply_all(False), 20, stream)
    roof_us = 96 * total / (PEAK_HBM_GBS * 1e9) * 1e6
    return {"systems": len(its), "grids": list(work.keys()), "systems_per_grid": nr, "total_dofs": total,
            "batched_ms": round(t_batch, 3), "batched_mdofs": round(total / (t_batch * 1e-3) / 1e6, 2),
            "batched_graph_ms": round(t_batch_graph, 3),
            "grid_by_grid_ms": round(t_grid, 3), "one_by_one_ms": round(t_one, 3),
            "iterations_min_max": [min(its), max(its)],
            "max_true_rel_res": float(f"{max(i['true_rel_res'] for i in info):.3e}"),
            "apply_fp64": {"concurrent_us": round(ms_conc * 1e3, 1), "grid_by_grid_us": round(ms_seq * 1e3, 1),
                           "mdofs": round(total / (ms_conc * 1e-3) / 1e6, 1), "hbm_roof_us": round(roof_us, 1),
                           "frac": round(roof_us / (ms_conc * 1e3), 4)}}


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


def shifted_section(stream, reps=5):
    """The 2D Gaussian-potential step (right-hand side with lifting + FP64 PCG to 1e-8) with the
    preconditioner built for S + c, c = mean of V (STFD_SHIFT_MEAN_POTENTIAL), and the 3D p = 3 48^4
    harmonic solve with it; the headline step keeps the V-free preconditioner of the workload."""
    import torch
    from paper_2311_18461_amd import inputs, stfd
    dev = torch.device("cuda:0")
    out = {}
    w = inputs.gaussian_potential_2d_workload(0)
    ks = [w.knots_s()] * 2
    prob = stfd.Problem(w.knots_t(), ks, w.p, w.p, w.T, w.nu, V_quad=stfd.sample_on_quad_grid(w.potential, ks, w.p),
                        precond_shift=stfd.SHIFT_MEAN_POTENTIAL)
    u0 = torch.from_numpy(prob.sample_space(w.u0)).to(dev)
    f = torch.empty(prob.N, dtype=torch.complex128, device=dev)
    u = torch.empty_like(f)

    def step():
        prob.load_vector(f, u0_q=u0, stream=stream)
        return prob.pcg_solve(f, u, rtol=1e-8, maxit=1000, stream=stream)
    step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        rc, info = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) / reps * 1e3
    out["gauss2d_p3_n64"] = {"shift": round(prob.precond_shift, 6), "step_ms": round(ms, 3),
                             "mdofs": round(prob.N / (ms * 1e-3) / 1e6, 2), "iterations": info[0]["iters"],
                             "true_rel_res": float(f"{info[0]['true_rel_res']:.3e}")}
    prob.close()
    w = inputs.harmonic_3d_workload(0, n_el=48, p=3, with_potential=True)
    ks = [w.knots_s()] * 3
    prob = stfd.Problem(w.knots_t(), ks, 3, 3, w.T, w.nu, V_quad=stfd.sample_on_quad_grid(w.potential, ks, 3),
                        precond_shift=stfd.SHIFT_MEAN_POTENTIAL, autotune=True)
    f = torch.empty(prob.N, dtype=torch.complex128, device=dev)
    u = torch.empty_like(f)
    prob.load_vector(f, u0_q=torch.from_numpy(prob.sample_space(w.u0)).to(dev), stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, info = prob.pcg_solve(f, u, rtol=1e-8, maxit=1000, stream=stream)
    torch.cuda.synchronize()
    out["harm3d_p3_n48"] = {"shift": round(prob.precond_shift, 6),
                            "pcg_ms": round((time.perf_counter() - t1) * 1e3, 2), "iterations": info[0]["iters"],
                            "true_rel_res": float(f"{info[0]['true_rel_res']:.3e}")}
    prob.close()
    return out


def ultraweak_section(stream, reps=5):
    """The 2D Gaussian-potential workload solved by the ultraweak method (Section 4.4): final-condition
    test space, load vector (f, B_I) + i (u_0, B_I(0)) with no lifting, FP64 PCG to 1e-8 (same
    preconditioner and kernels as the least-squares solve)."""
    import torch
    from paper_2311_18461_amd import inputs, stfd
    dev = torch.device("cuda:0")
    w = inputs.gaussian_potential_2d_workload(0)
    ks = [w.knots_s()] * 2
    t0 = time.perf_counter()
    prob = stfd.Problem(w.knots_t(), ks, w.p, w.p, w.T, w.nu, V_quad=stfd.sample_on_quad_grid(w.potential, ks, w.p),
                        time_condition=stfd.TIME_FINAL)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    u0 = torch.from_numpy(prob.sample_space(w.u0)).to(dev)
    f = torch.empty(prob.N, dtype=torch.complex128, device=dev)
    z = torch.empty_like(f)

    def step():
        prob.load_vector(f, u0_q=u0, stream=stream)
        return prob.pcg_solve(f, z, rtol=1e-8, maxit=1000, stream=stream)
    step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        rc, info = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) / reps * 1e3
    prob.close()
    return {"workload": "2D p=3 64^3 8-Gaussian potential, wave-packet u_0, f = 0 (ultraweak method)",
            "n_dof_free": prob.N, "setup_s": round(setup_s, 3), "rhs_and_pcg_ms": round(ms, 3),
            "mdofs": round(prob.N / (ms * 1e-3) / 1e6, 2), "iterations": info[0]["iters"], "converged": rc == 0,
            "true_rel_res": float(f"{info[0]['true_rel_res']:.3e}")}


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
        prob = stfd.Problem(w.knots_t(), ks, p, p, w.T, w.nu, V_quad=stfd.sample_on_quad_grid(w.potential, ks, p),
                            autotune=True)
        torch.cuda.synchronize()
        row = {"n_dof_free": prob.N, "setup_s": round(time.perf_counter() - t0, 2), "tuning": prob.get_tuning()}
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
        # the fused last-direction launch (x_d products and time solves in one kernel), where it
        # fits: apply time and agreement with the separate launches the tuning kept
        t = row["tuning"]
        if t["fused_segment_length"]:
            fz = {}
            for prec in ("fp64", "fp32"):
                prob.set_fused_time(True)
                prob.apply_preconditioner(r, z, precision=prec, stream=stream)
                ms = time_events(lambda: prob.apply_preconditioner(r, z, precision=prec, stream=stream), 10, stream)
                prob.set_fused_time(t["fused_time"])
                zs = torch.empty_like(z)
                prob.apply_preconditioner(r, zs, precision=prec, stream=stream)
                d_sep = float(torch.max(torch.abs(z - zs)) / torch.max(torch.abs(zs)))
                fz[prec] = {"apply_ms": round(ms, 4), "max_rel_diff_vs_kept": float(f"{d_sep:.3e}")}
            row["fused_last_direction"] = {"segment_length": t["fused_segment_length"], **fz}
        row["matvec_ms"] = round(time_events(lambda: prob.matvec(r, z, stream=stream), 10, stream), 4)
        # FP64 mode products timed one by one (HIP events on the launch stream), and the whole apply
        # against its roof
        prob.timing_begin(capacity=6 * 10)
        for _ in range(10):
            prob.apply_preconditioner(r, z, precision="fp64", stream=stream)
        mp_ms, mp_n = prob.timing_end()
        n_s = prob.n_s[0]
        mp_us_bracketed = mp_ms / mp_n * 1e3
        mp_us = prob.time_mode_product(0, "fp64", 100, stream) * 1e3  # back-to-back launches
        row["mode_product_fp64"] = {"avg_launch_us": round(mp_us, 2), "avg_launch_us_bracketed": round(mp_us_bracketed, 2),
                                    "hbm_frac": round(32 * prob.N / (mp_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4),
                                    "algorithmic_tflops": round(4 * n_s * prob.N / (mp_us * 1e-6) / 1e12, 3)}
        row["fd_apply_roofline_fp64"] = fd_apply_roofline(prob.N, 3, n_s, p, row["fp64"]["apply_ms"] * 1e3)
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


def mode_product_roofline(N, n, avg_us):
    """HBM roofline of one FP64 mode product (read and write the complex FP64 tensor: 32 bytes per
    dof; 4 n flops per dof), with the MFMA work the counters measured for it."""
    bytes_alg = 32 * N
    achieved = bytes_alg / (avg_us * 1e-6) / 1e9
    mfma_tflops = MODE_PRODUCT_MFMA_FLOPS / (avg_us * 1e-6) / 1e12
    return {"bound": "hbm", "kernel": MODE_PRODUCT_KERNEL, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": MODE_PRODUCT_TRAFFIC_BYTES,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated)",
            "traffic_algorithmic": bytes_alg, "avg_launch_us": round(avg_us, 3),
            "algorithmic_flops": 4 * n * N,
            "mfma": {"flops_per_launch": MODE_PRODUCT_MFMA_FLOPS, "source": "SQ_INSTS_VALU_MFMA_MOPS_F64 x 512",
                     "achieved_tflops": round(mfma_tflops, 3), "peak_tflops": PEAK_FP64_TFLOPS,
                     "frac": round(mfma_tflops / PEAK_FP64_TFLOPS, 4)}}


def fd_apply_roofline(N, d, n_s, p, apply_us):
    """Whole FP64 FD apply against max(flops / FP64 peak, bytes / HBM) with the algorithmic work of
    Algorithm 1: 8 d n_s + 16 p + 4 flops and 96 bytes (three passes of complex FP64 intermediates)
    per dof."""
    flops = (8 * d * n_s + 16 * p + 4) * N
    t_roof = max(flops / (PEAK_FP64_TFLOPS * 1e12), 96 * N / (PEAK_HBM_GBS * 1e9))
    return {"apply_us": round(apply_us, 2), "flops": flops, "roof_us": round(t_roof * 1e6, 2),
            "frac": round(t_roof * 1e6 / apply_us, 4)}


def table2_section(stream, p=3, n_el=64):
    """Table 2's workload (traveling wave, 2D, T = 1, p = 3, 64 elements per direction, x0 = 0, tol
    1e-8): setup + right-hand side + PCG wall time on the GPU, beside the paper's serial figure."""
    import torch
    from paper_2311_18461_amd import inputs, stfd
    dev = torch.device("cuda:0")
    w = inputs.traveling_wave_workload(n_el, p)
    ks = [w.knots_s()] * 2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob = stfd.Problem(w.knots_t(), ks, p, p, w.T, w.nu)
    t_setup = time.perf_counter() - t0
    f_q = torch.from_numpy(prob.sample_spacetime(w.f)).to(dev)
    u0_q = torch.from_numpy(prob.sample_space(w.u0)).to(dev)
    faces = [torch.from_numpy(a).to(dev) for a in prob.sample_faces(w.dirichlet)]
    fb = torch.empty(prob.N, dtype=torch.complex128, device=dev)
    u = torch.empty_like(fb)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prob.load_vector(fb, f_q=f_q, u0_q=u0_q, dirichlet_q=faces, stream=stream)
    rc, info = prob.pcg_solve(fb, u, rtol=1e-8, maxit=200, stream=stream)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t1
    prob.close()
    return {"workload": f"traveling wave (Table 2), 2D, p={p}, n_el={n_el}", "n_dof_free": prob.N,
            "iterations": info[0]["iters"], "setup_s": round(t_setup, 3),
            "rhs_and_pcg_s": round(t_solve, 4), "total_s": round(t_setup + t_solve, 3),
            "paper": {"iterations": 8, "total_s": 4.7142,
                      "hardware": "Intel Core i5-1035G1, one thread at 1 GHz, MATLAB (Table 2)"}}


def cpu_baseline(w, iterations, budget_s=25.0):
    """The oracle (FP64 NumPy/SciPy) on a bounded sample of the same workload: the right-hand side
    with lifting once, then 5 samples of 8 PCG iterations, the step time scaled to `iterations`
    iterations (the GPU solve's count); on all host cores and with one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.operators import FastDiagonalization, Problem as OProblem
    from oracle.pcg import pcg
    from oracle.rhs import SpaceTimeBasis, assemble_rhs
    ks = [w.knots_s()] * 2
    ref = OProblem(w.knots_t(), ks, w.p, w.p, w.nu, w.potential)
    fd = FastDiagonalization(ref)
    stb = SpaceTimeBasis(w.knots_t(), ks, w.p, w.p)

    def sample(n_samples):
        t0 = time.perf_counter()
        fb, _ = assemble_rhs(stb, w.nu, u0=w.u0, V=w.potential)
        t_rhs = time.perf_counter() - t0
        per_it = []
        for _ in range(n_samples):
            t1 = time.perf_counter()
            _, info = pcg(ref.matvec, fd.apply, fb, tol=1e-8, maxit=8)
            per_it.append((time.perf_counter() - t1) / info["iters"])
        return t_rhs, float(np.median(per_it)), per_it

    t_start = time.perf_counter()
    t_rhs, t_it, per_it = sample(5)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    step = t_rhs + iterations * t_it
    out = {"value": ref.N / step / 1e6, "unit": "Mdof/s", "cores": int(threads), "kind": "oracle",
           "sample": f"right-hand side with lifting once ({t_rhs:.2f} s) + 5 samples of 8 FP64 PCG iterations "
                     f"(median {t_it * 1e3:.1f} ms per iteration, samples {[round(x * 1e3, 1) for x in per_it]} ms), "
                     f"step scaled to {iterations} iterations: {step:.2f} s"}
    if time.perf_counter() - t_start < budget_s * 0.5:
        with threadpool_limits(limits=1):
            t_rhs1, t_it1, per_it1 = sample(3)
        step1 = t_rhs1 + iterations * t_it1
        out["one_thread"] = {"value": ref.N / step1 / 1e6, "cores": 1,
                             "sample": f"right-hand side {t_rhs1:.2f} s + 3 samples of 8 iterations (median "
                                       f"{t_it1 * 1e3:.1f} ms per iteration), scaled to {iterations} iterations: "
                                       f"{step1:.2f} s"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D precision section")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--profile", nargs="?", const="2d", choices=["2d", "3d48", "3d32", "long1d"],
                    help="short run for rocprofv3 on one workload (2d: the 2D p=3 64^3 Gaussian-potential step; "
                         "3d48 / 3d32: the 3D harmonic workloads p=3 48^4 / p=4 32^4): one solve, 20 applies per "
                         "precision (3D: and 20 FP64 applies with the fused last-direction launch), 20 matvecs, "
                         "and a device copy of known size (64 MiB read + 64 MiB written) to calibrate FETCH_SIZE / "
                         "WRITE_SIZE; long1d: the Section 6.1 high-mode series on 512 x 1024 elements, p = 4 "
                         "(long axes), solved to 1e-10")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU per process; --gpus must be 1",
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
        if args.profile == "long1d":
            prob.close()
            p, n = 4, 512
            series = inputs.HighModeSeries1D(625)
            prob = stfd.Problem(inputs.uniform_open_knots(2 * n, p), [inputs.uniform_open_knots(n, p)], p, p, 2.0, 1.0)
            N = prob.N
            f = torch.empty(N, dtype=torch.complex128, device=dev)
            u = torch.empty_like(f)
            fq = series.f_grid(prob.quad[0][0], prob.quad[1][0]).ravel()
            prob.load_vector(f, f_q=torch.from_numpy(fq).to(dev), stream=stream)
            rc, info = prob.pcg_solve(f, u, rtol=1e-10, maxit=1000, stream=stream)
        elif args.profile != "2d":
            prob.close()
            n_el, p = (48, 3) if args.profile == "3d48" else (32, 4)
            w3 = inputs.harmonic_3d_workload(0, n_el=n_el, p=p, with_potential=True)
            ks = [w3.knots_s()] * 3
            prob = stfd.Problem(w3.knots_t(), ks, p, p, w3.T, w3.nu,
                                V_quad=stfd.sample_on_quad_grid(w3.potential, ks, p))
            N = prob.N
            f = torch.empty(N, dtype=torch.complex128, device=dev)
            u = torch.empty_like(f)
            prob.load_vector(f, u0_q=torch.from_numpy(prob.sample_space(w3.u0)).to(dev), stream=stream)
            rc, info = solve("fp64")
        else:
            step()
            rc, info = step()
        r = torch.from_numpy(inputs.random_complex(N, 2998)).to(dev)
        s = torch.empty_like(r)
        for prec in ("fp64", "fp32", "bf16"):
            for _ in range(20):
                prob.apply_preconditioner(r, s, precision=prec, stream=stream)
        if args.profile != "2d" and prob.get_tuning()["fused_segment_length"]:
            # the fused last-direction launch (off by default): 20 FP64 applies
            prob.set_fused_time(True)
            for _ in range(20):
                prob.apply_preconditioner(r, s, precision="fp64", stream=stream)
            prob.set_fused_time(False)
        for _ in range(20):
            prob.matvec(r, s, stream=stream)
        src = torch.ones(8 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": args.profile, "n_dof_free": N, "iterations": info[0]["iters"],
                          "copy_bytes": src.numel() * 8}))
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
    # the dominant kernel: every FP64 mode-product launch of 50 applies timed with HIP events on the
    # launch stream (library timing hooks)
    prob.timing_begin(capacity=4 * 50)
    for _ in range(50):
        prob.apply_preconditioner(r, s, precision="fp64", stream=stream)
    mp_total_ms, mp_launches = prob.timing_end()
    mp_us = mp_total_ms / mp_launches * 1e3
    mp_b2b_us = prob.time_mode_product(0, "fp64", 500, stream) * 1e3
    roofline = mode_product_roofline(N, 65, mp_b2b_us)
    roofline["avg_launch_us_bracketed"] = round(mp_us, 3)
    roofline["fd_apply"] = fd_apply_roofline(N, 2, 65, w.p, apply_ms["fp64"] * 1e3)
    roofline["matvec_us"] = round(matvec_ms * 1e3, 2)

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
    out["table2_p3_n64"] = table2_section(stream)
    out["ultraweak"] = ultraweak_section(stream)
    out["mean_potential_preconditioner"] = shifted_section(stream)
    out["batched"] = batched_section(dev, stream)
    out["warm_start"] = warmstart_section(stream)
    if not args.no_3d:
        out["precision_3d"] = precision_3d_section(stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, int(np.median(iters)))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
