"""Pins of the C/OpenMP oracle product (the benchmark's timed CPU baseline):
it equals the numpy oracle's block-order product (eq. 4) on the same stored
values for H, UH and H^2, with one thread and with all of them, and it
reproduces the closed forms of the constant and identity kernels."""
import numpy as np
import pytest

from conftest import cached
from oracle import mvm, omp, stored, trees
from synth import (KERNEL_CONST, KERNEL_IDENTITY, KERNEL_LAPLACE, compress_h, gaussian_vector, sphere_points,
                   to_h2, to_uh)


def case(n, kernel, eps, seed):
    def make():
        p = sphere_points(n, seed)
        st = trees.build_structure(p)
        h = compress_h(p, kernel, st, eps, method="svd")
        return st, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    return cached(("omp-case", n, kernel, eps, seed), make)


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("threads", [1, 0])
def test_omp_equals_block_order(fmt, threads):
    n = 2048
    st, vals = case(n, KERNEL_LAPLACE, 1e-8, 1001)
    x, y = gaussian_vector(n, 2001), gaussian_vector(n, 3001)
    ref = stored.product(st, fmt, vals[fmt], -0.5, x, y)
    out, used = omp.Prepared(st, fmt, vals[fmt]).product(-0.5, x, y, threads)
    assert used >= 1 and (threads != 1 or used == 1)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref - y) < 1e-13


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_omp_stored_values_and_closed_forms(fmt):
    """Compressed storage (the dequantised values) and two closed forms:
    constant kernel y_i = y_in,i + a (sum x - x_i), identity y = y_in + a x
    (every admissible block has rank 0, so the bases are empty)."""
    n = 1500
    st, vals = case(n, KERNEL_LAPLACE, 1e-6, 77)
    x, y = gaussian_vector(n, 78), gaussian_vector(n, 79)
    sv = stored.stored_values(st, fmt, vals[fmt], dense="valr", diag="valr", factor="valr", eps=1e-6)
    ref = stored.product(st, fmt, sv, 1.0, x, y)
    assert np.linalg.norm(omp.product(st, fmt, sv, 1.0, x, y) - ref) / np.linalg.norm(ref - y) < 1e-13
    st, vals = case(n, KERNEL_CONST, 1e-10, 80)
    out = omp.product(st, fmt, vals[fmt], 0.25, x, y)
    assert np.allclose(out, y + 0.25 * (x.sum() - x), rtol=0, atol=1e-9)
    st, vals = case(n, KERNEL_IDENTITY, 1e-10, 81)
    out = omp.product(st, fmt, vals[fmt], 2.0, x, y)
    assert np.allclose(out, y + 2.0 * x, rtol=0, atol=1e-13)


def test_triad_probe_runs():
    gbs, used = omp.triad_gbs(nbytes=3e7, reps=2)
    assert gbs > 0.1 and used >= 1
