"""Mesh-size edge cases on every stage kernel, through the C ABI, against the
FP64 oracle: a single element (every face on the PEC wall, the grid's other
vertices unused), exactly one 64-element tile (no padding), and one tile plus
one element (the smallest ragged tail), in 2D and 3D.  Sub-meshes are the
first k elements of a conforming grid, which is again conforming (the cut
faces become walls).  Tolerances are those of the full-size parity tests of
each arithmetic."""

import copy

import numpy as np
import pytest

import oracle
from paper_1304_5546_amd import dgw, inputs

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_bf16": 1e-4, "split_fp16": 1e-5, "fp64": 1e-12}
KERNELS_2D = [("fp32", 1), ("fp32", 2), ("fp32", 3), ("fp32", 4), ("split_bf16", 0), ("split_fp16", 0),
              ("fp64", 1), ("fp64", 3)]


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def first_elements(m, k):
    s = copy.copy(m)
    s.elem_verts = np.ascontiguousarray(m.elem_verts[:k])
    return s


@pytest.mark.parametrize("k", [1, 64, 65])
@pytest.mark.parametrize("N", [1, 4, 8])
def test_2d_sizes_every_kernel(k, N):
    m = first_elements(inputs.tri_grid(6, seed=3, permute=True), k)
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, N)
    op = oracle.Maxwell2D(d, 1.0)
    q = np.random.default_rng(100 * k + N).standard_normal((3, k, d.x.shape[1]))
    want = op.rhs(q)
    for prec, kern in KERNELS_2D:
        with dgw.Solver(m, N, prec=prec, kernel=kern) as s:
            err = rel(s.rhs(q), want)
            print(f"2D K={k} N={N} {prec} kernel {kern}: {err:.2e}")
            assert err < TOL[prec], (prec, kern)


@pytest.mark.parametrize("k", [1, 64, 65])
@pytest.mark.parametrize("N", [1, 4])
def test_3d_sizes(k, N):
    m = first_elements(inputs.tet_grid(3, seed=2, permute=True), k)
    d = oracle.Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, N)
    op = oracle.Maxwell3D(d, 1.0)
    q = np.random.default_rng(100 * k + N).standard_normal((6, k, d.x.shape[1]))
    want = op.rhs(q)
    for prec in ("fp32", "split_bf16"):
        with dgw.Solver(m, N, prec=prec) as s:
            err = rel(s.rhs(q), want)
            print(f"3D K={k} N={N} {prec}: {err:.2e}")
            assert err < TOL[prec], prec


def test_single_element_steps_and_energy():
    """One triangle closed by PEC walls, 50 steps of every 2D arithmetic
    from a smooth state against the oracle's LSRK run; the upwind flux does
    not let the energy grow."""
    m = first_elements(inputs.tri_grid(6, seed=3, permute=True), 1)
    N = 5
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, N)
    op = oracle.Maxwell2D(d, 1.0)
    dt = oracle.cfl_dt(d, N)
    q0 = oracle.cavity_mode_2d(d.x, d.y, 0.0, 1, 1)
    want = op.run(q0, dt, 50)
    assert op.energy(want) <= op.energy(q0)
    for prec in ("fp32", "split_bf16", "split_fp16", "fp64"):
        with dgw.Solver(m, N, prec=prec) as s:
            s.set_fields(q0)
            s.advance_steps(50, dt)
            err = rel(s.get_fields(), want)
            print(f"single triangle 50 steps {prec}: {err:.2e}")
            assert err < TOL[prec], prec
