"""The byte model that prices the whole run against the HBM roofline (bench.py), checked
against hand-counted cases: one Arnoldi step, a cycle boundary, and a full Newton
iteration built term by term from the per-kernel formulas."""
import importlib.util
import os

import pytest

_spec = importlib.util.spec_from_file_location("bench", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def test_arnoldi_bytes_count_each_step_and_restart():
    # j = 0: 32 (0 + 1) + 64
    assert bench.arnoldi_bytes_per_cell(1) == 96.0
    # j = 0, 1, 2
    assert bench.arnoldi_bytes_per_cell(3) == 96.0 + 128.0 + 160.0
    # 32 steps in cycles of 30: j = 0..29 then j = 0, 1
    full = sum(32.0 * (j + 1) + 64.0 for j in range(30))
    assert bench.arnoldi_bytes_per_cell(32, m=30) == pytest.approx(full + 96.0 + 128.0)


def test_newton_iteration_bytes_from_the_kernel_formulas():
    nnz, omega, sp = 24, 1.25, 8
    k = 4   # GMRES iterations of the one Newton iteration; one step
    b = bench.step_bytes_per_cell(newton=1, gmres=k, steps=1, nnz=nnz, omega=omega, sp=sp)
    b_ras = omega * 16 + omega * nnz * sp + 16
    want = (2 * 48 + (32 + 8 * nnz) + omega * nnz * (8 + sp)
            + k * ((8 * nnz + 32) + b_ras) + sum(32 * (j + 1) + 64 for j in range(k)) + 16 * (k + 1))
    assert b == pytest.approx(want)
    # three Newton iterations share the step's one factorisation
    b3 = bench.step_bytes_per_cell(newton=3, gmres=3 * k, steps=1, nnz=nnz, omega=omega, sp=sp)
    assert b3 == pytest.approx(3 * (want - omega * nnz * (8 + sp)) + omega * nnz * (8 + sp))
