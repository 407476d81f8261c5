"""Oracle parity at the full benchmark sizes, in the launch configuration the
benchmark times (persistent grids in which every work-group or wave walks
many tiles, so the multi-tile loops, the double-buffered producer/consumer
hand-over and the prefetch of the next tile's operands are all exercised).

  * 512 x 512 grid (524288 triangles), N = 7: one LSRK4 step of the cavity
    mode (2,3) and one right-hand side of random data, for FP32 (the
    fused-operand kernel, the order-7 default), split-BF16 and split-FP16.
  * 48^3 x 6 = 663552 tetrahedra, N = 4: one right-hand side of random data
    for the FP32 and split-BF16 3D kernels; one LSRK4 step of the (1,1,1)
    mode on 24^3 x 6 = 82944 tetrahedra (several work units per wave).

Each comparison reports the global relative L2 and the worst element's
max-abs error relative to the largest oracle value, and asserts both.
Tolerances: FP32 1e-6 (L2) / 1e-5 (element max) after one step, split-BF16
1e-4 / 1e-3, split-FP16 1e-5 / 1e-4; a right-hand side of random data (whose
entries reach ~N^2/h) 1e-5 / 1e-4 (FP32, FP16) and 1e-4 / 1e-3 (BF16).
"""

import numpy as np
import pytest

import oracle
from oracle.maxwell import cfl_dt
from paper_1304_5546_amd import dgw, inputs

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

STEP_TOL = {"fp32": (1e-6, 1e-5), "split_bf16": (1e-4, 1e-3), "split_fp16": (1e-5, 1e-4)}
RHS_TOL = {"fp32": (1e-5, 1e-4), "split_bf16": (1e-4, 1e-3), "split_fp16": (1e-5, 1e-4)}


def compare(got, want, label):
    """Global relative L2 and worst per-element max-abs error (relative to
    max |want|); prints both with the worst element's index."""
    l2 = float(np.linalg.norm((got - want).ravel()) / np.linalg.norm(want.ravel()))
    per_el = np.abs(got - want).max(axis=(0, 2))         # [K]
    k = int(np.argmax(per_el))
    emax = float(per_el[k] / np.abs(want).max())
    print(f"{label}: rel L2 {l2:.2e}, worst element {k} max-abs {emax:.2e}", flush=True)
    return l2, emax


@pytest.fixture(scope="module")
def c3():
    print("C3 oracle set-up (524288 triangles, N = 7)", flush=True)
    m = inputs.tri_grid(512, seed=3)
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, 7)
    op = oracle.Maxwell2D(d)
    dt = cfl_dt(d, 7)
    q0 = oracle.cavity_mode_2d(d.x, d.y, 0.0, 2, 3)
    q1, res = q0.copy(), np.zeros_like(q0)
    op.lsrk4_step(q1, res, dt)
    rng = np.random.default_rng(3)
    qr = rng.standard_normal(q0.shape)
    return dict(m=m, dt=dt, q0=q0, q1=q1, qr=qr, rhs=op.rhs(qr))


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
def test_c3_full_size_one_step_and_rhs(c3, prec):
    with dgw.Solver(c3["m"], 7, prec=prec) as s:
        if prec == "fp32":
            assert s.info()["kernel"] == 2      # the fused-operand kernel is the order-7 default
        s.set_fields(c3["q0"])
        s.advance_steps(1, c3["dt"])
        l2, emax = compare(s.get_fields(), c3["q1"], f"C3 {prec} one step")
        assert l2 < STEP_TOL[prec][0] and emax < STEP_TOL[prec][1]
        l2, emax = compare(s.rhs(c3["qr"]), c3["rhs"], f"C3 {prec} rhs of random data")
        assert l2 < RHS_TOL[prec][0] and emax < RHS_TOL[prec][1]


@pytest.fixture(scope="module")
def c5():
    print("C5 oracle set-up (663552 tetrahedra, N = 4)", flush=True)
    m = inputs.tet_grid(48, seed=5)
    d = oracle.Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, 4)
    op = oracle.Maxwell3D(d)
    rng = np.random.default_rng(5)
    qr = rng.standard_normal((6, d.K, d.Np))
    return dict(m=m, qr=qr, rhs=op.rhs(qr))


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_c5_full_size_rhs(c5, prec):
    with dgw.Solver(c5["m"], 4, prec=prec) as s:
        l2, emax = compare(s.rhs(c5["qr"]), c5["rhs"], f"C5 {prec} rhs of random data")
        assert l2 < RHS_TOL[prec][0] and emax < RHS_TOL[prec][1]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_3d_one_step_many_units(prec):
    m = inputs.tet_grid(24, seed=8, permute=True)
    d = oracle.Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, 4)
    op = oracle.Maxwell3D(d)
    dt = cfl_dt(d, 4)
    q0 = oracle.cavity_mode_3d(d.x, d.y, d.z, 0.0)
    q1, res = q0.copy(), np.zeros_like(q0)
    op.lsrk4_step(q1, res, dt)
    with dgw.Solver(m, 4, prec=prec) as s:
        s.set_fields(q0)
        s.advance_steps(1, dt)
        l2, emax = compare(s.get_fields(), q1, f"3D 82944 tets {prec} one step")
    assert l2 < STEP_TOL[prec][0] and emax < STEP_TOL[prec][1]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
def test_material_order7_multi_tile_one_step(prec):
    """Order 7 on a material mesh large enough that every work-group of the
    default launch walks two tiles (128 x 128 grid, 32768 triangles, 512
    tiles): the material forms of the fused-operand and split kernels,
    including the row-major update through the LDS sub-tile, against one
    oracle LSRK4 step of random data with eps/mu jumps."""
    m = inputs.tri_grid(128, seed=11, permute=True)
    m.eps = inputs.disk_inclusion_eps(m, (0.1, -0.2), 0.45)
    m.mu = np.where(np.arange(m.K) % 3 == 0, 1.5, 1.0)
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, 7, eps=m.eps, mu=m.mu)
    op = oracle.Maxwell2D(d, 1.0)
    dt = cfl_dt(d, 7)
    q0 = np.random.default_rng(11).standard_normal((3, d.K, d.Np))
    q1, res = q0.copy(), np.zeros_like(q0)
    op.lsrk4_step(q1, res, dt)
    with dgw.Solver(m, 7, prec=prec) as s:
        if prec == "fp32":
            assert s.info()["kernel"] == 2
        s.set_fields(q0)
        s.advance_steps(1, dt)
        l2, emax = compare(s.get_fields(), q1, f"material N=7 32768 triangles {prec} one step")
    assert l2 < STEP_TOL[prec][0] and emax < STEP_TOL[prec][1]
