"""Sweep of the setup-time autotune over the benchmark workloads: the tile table.

For every key (d, n_s, n_t, p) of the workloads and every precision of the FD apply, sets the
problem up twice (heuristic launch shapes, and autotune = 1, which times the candidate shapes on
the device), prints the chosen shapes (mode-product row groups per direction, time-solve segment
length and transfer mode, whether the fused last-direction launch was kept) and the apply time of
both, with the fused launch's own apply time, as a Markdown table.

    python -m paper_2311_18461_amd.autotune_sweep [--reps 20]
"""
from __future__ import annotations

import argparse

import numpy as np

from . import inputs, stfd

# (label, d, n_el, p, potential)
WORKLOADS = [("2D Gaussian potential", 2, 64, 3, "gauss")] + \
    [(f"2D batched grid {n}^3", 2, n, 3, None) for n in inputs.BATCH_GRIDS[:-1]] + \
    [("3D harmonic", 3, 48, 3, "harm"), ("3D harmonic", 3, 32, 4, "harm")]


def _potential(kind, d):
    if kind == "gauss":
        return inputs.gaussian_potential(d, 2000)
    if kind == "harm":
        return inputs.harmonic_potential(d, 3000)
    return None


def _form(t):
    """tables: L, 1/D and transfers read; transfers: L and 1/D read; factor: all computed."""
    if t["time_factors_in_kernel"]:
        return "factor"
    return "transfers" if t["time_transfers_in_kernel"] else "tables"


def _apply_us(pr, prec, reps, torch):
    r = torch.from_numpy(inputs.random_complex(pr.N, 1)).to("cuda")
    z = torch.empty_like(r)
    s = torch.cuda.current_stream()
    pr.apply_preconditioner(r, z, precision=prec)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        pr.apply_preconditioner(r, z, precision=prec)
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) / reps * 1e3


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    print("| workload | d | n_s | n_t | p | precision | row groups (heuristic -> tuned) | time segment "
          "(heuristic -> tuned) | time-solve form (heuristic -> tuned) | apply us heuristic | "
          "apply us tuned | fused last direction: tuned, us | tune ms |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|---|")
    for label, d, n_el, p, kind in WORKLOADS:
        V = _potential(kind, d)
        kt = inputs.uniform_open_knots(n_el, p)
        ks = [inputs.uniform_open_knots(n_el, p)] * d
        Vq = stfd.sample_on_quad_grid(V, ks, p) if V is not None else None
        heur = stfd.Problem(kt, ks, p, p, 1.0, 1.0, V_quad=Vq)
        tuned = stfd.Problem(kt, ks, p, p, 1.0, 1.0, V_quad=Vq, autotune=True)
        th, tt = heur.get_tuning(), tuned.get_tuning()
        for prec in ("fp64", "fp32", "bf16"):
            uh = _apply_us(heur, prec, args.reps, torch)
            ut = _apply_us(tuned, prec, args.reps, torch)
            fz = "n/a"
            if tt["fused_segment_length"] and prec != "bf16":
                # the fused launch (segment length, form) on the tuned handle, whether kept or not
                tuned.set_fused_time(True)
                uf = _apply_us(tuned, prec, args.reps, torch)
                tuned.set_fused_time(tt["fused_time"])
                fz = (f"{'on' if tt['fused_time'] else 'off'} (segment {tt['fused_segment_length']}, "
                      f"{'factor' if tt['fused_factors_in_kernel'] else 'tables'}), {uf:.1f}")
            print(f"| {label} | {d} | {heur.n_s[0]} | {heur.n_t} | {p} | {prec} | "
                  f"{th['mode_product_row_groups'][prec]} -> {tt['mode_product_row_groups'][prec]} | "
                  f"{th['time_segment_length']} -> {tt['time_segment_length']} | "
                  f"{_form(th)} -> {_form(tt)} | "
                  f"{uh:.1f} | {ut:.1f} | {fz} | {tt['tune_ms']:.0f} |", flush=True)
        heur.close()
        tuned.close()


if __name__ == "__main__":
    main()
