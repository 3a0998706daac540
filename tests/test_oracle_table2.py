"""Table 2 of the paper: iteration counts of P-hat-preconditioned CG (traveling wave, 2D + time).

The oracle must reproduce the printed counts within one iteration (the lifting
of the boundary data and the residual norm are not specified by the paper).
"""
import json
import os

import numpy as np
import pytest

from oracle.operators import FastDiagonalization, Problem
from oracle.pcg import pcg
from oracle.rhs import SpaceTimeBasis, assemble_rhs
from paper_2311_18461_amd.inputs import traveling_wave_workload

CASES = [(p, n) for p in (2, 3, 4) for n in (8, 16, 32)] + [(3, 64)]
SLOW = [(2, 64), (4, 64)]


def _iterations(p, n):
    w = traveling_wave_workload(n, p)
    ks = [w.knots_s()] * 2
    pr = Problem(w.knots_t(), ks, p, p, w.nu)
    stb = SpaceTimeBasis(w.knots_t(), ks, p, p)
    fb, _ = assemble_rhs(stb, w.nu, f=w.f, u0=w.u0, dirichlet=w.dirichlet)
    _, info = pcg(pr.matvec, FastDiagonalization(pr).apply, fb, tol=1e-8, maxit=200)
    assert info["converged"] and info["true_rel_res"] <= 1.2e-8
    return info["iters"]


def _expected(golden_dir, p, n):
    ref = json.load(open(os.path.join(golden_dir, "table2_iterations.json")))
    return ref["iterations"][str(p)][ref["n_el"].index(n)]


@pytest.mark.parametrize("p,n", CASES)
def test_table2_iterations(golden_dir, p, n):
    assert abs(_iterations(p, n) - _expected(golden_dir, p, n)) <= 1


@pytest.mark.slow
@pytest.mark.parametrize("p,n", SLOW)
def test_table2_iterations_n64(golden_dir, p, n):
    assert abs(_iterations(p, n) - _expected(golden_dir, p, n)) <= 1
