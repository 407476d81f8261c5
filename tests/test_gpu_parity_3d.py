"""GPU parity of the fused 3D stage kernel (tetrahedra, 6 fields, 4 faces with
orientation table) against the FP64 oracle, through the C ABI."""

import numpy as np
import pytest

import oracle
from oracle.maxwell import cfl_dt
from paper_1304_5546_amd import dgw, inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _setup(m, N, alpha=1.0):
    d = oracle.Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, N)
    return d, oracle.Maxwell3D(d, alpha), dgw.Solver(m, N, alpha=alpha)


@pytest.mark.parametrize("n,N,seed,permute,alpha", [
    (2, 1, 1, False, 1.0),   # 48 tets: one ragged tile
    (2, 2, 2, True, 1.0),
    (3, 3, 3, True, 1.0),    # 162 tets: 3 tiles, ragged tail
    (3, 4, 4, True, 1.0),
    (2, 4, 5, False, 0.0),   # central flux
])
def test_single_rhs_parity_3d(n, N, seed, permute, alpha):
    m = inputs.tet_grid(n, seed=seed, permute=permute)
    d, op, sol = _setup(m, N, alpha)
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(sol.shape)
    err = rel(sol.rhs(q), op.rhs(q))
    print(f"3D rhs parity n={n} N={N} K={m.K}: {err:.2e}")
    assert err < 1e-5
    q = oracle.cavity_mode_3d(d.x, d.y, d.z, 0.2)
    err2 = rel(sol.rhs(q), op.rhs(q))
    print(f"   smooth: {err2:.2e}")
    assert err2 < 1e-5


def test_steps_parity_3d_and_reductions():
    m = inputs.tet_grid(3, seed=6, permute=True)
    d, op, sol = _setup(m, 3)
    dt = cfl_dt(d, 3)
    assert abs(sol.cfl_dt() / dt - 1) < 1e-13
    q0 = oracle.cavity_mode_3d(d.x, d.y, d.z, 0.0)
    sol.set_fields(q0)
    e0 = sol.energy()
    sol.advance_steps(30, dt)
    got = sol.get_fields()
    want = op.run(q0, dt, 30)
    err = rel(got, want)
    print(f"3D 30 steps: {err:.2e}")
    assert err < 1e-5
    assert abs(sol.energy() / op.energy(got) - 1) < 1e-12
    assert sol.energy() < e0
    ex = oracle.cavity_mode_3d(d.x, d.y, d.z, 30 * dt)
    assert abs(sol.cavity_error(1, 1, 1, 30 * dt) / op.rel_l2(got, ex) - 1) < 1e-9
    # device initialisation of the (1,1,1) mode matches the closed form
    sol.set_cavity_mode(1, 1, 1)
    assert np.abs(sol.get_fields() - q0).max() < 1e-7


def test_3d_full_size_vs_closed_form():
    """48^3 cubes x 6 = 663552 tetrahedra, N = 4, mode (1,1,1), to t = 1 at
    the CFL step: FP32 GPU result against the closed-form mode."""
    m = inputs.tet_grid(48, seed=5)
    with dgw.Solver(m, 4) as s:
        s.set_cavity_mode(1, 1, 1)
        n = s.advance(1.0)
        err = s.cavity_error(1, 1, 1, 1.0)
        print(f"3D 663552 tets to t=1 in {n} steps: rel L2 vs closed form {err:.2e}")
        assert err < 1e-5


@pytest.mark.parametrize("n,N,seed,permute", [
    (2, 1, 1, False),
    (2, 2, 2, True),
    (3, 3, 3, True),   # 162 tets: 3 tiles, ragged tail
    (3, 4, 4, True),
])
def test_split_bf16_rhs_parity_3d(n, N, seed, permute):
    """Split-BF16 3D stage: one right-hand side against the oracle.  The
    operands carry ~2^-17 relative error per hi+lo split and the dropped
    lo*lo term ~2^-18; with the cancellation of the reference derivatives
    we allow 1e-4 (random data) and 5e-4 (smooth data)."""
    m = inputs.tet_grid(n, seed=seed, permute=permute)
    d = oracle.Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, N)
    op = oracle.Maxwell3D(d, 1.0)
    sol = dgw.Solver(m, N, prec="split_bf16")
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(sol.shape)
    err = rel(sol.rhs(q), op.rhs(q))
    q2 = oracle.cavity_mode_3d(d.x, d.y, d.z, 0.2)
    err2 = rel(sol.rhs(q2), op.rhs(q2))
    print(f"3D split_bf16 rhs n={n} N={N} K={m.K}: random {err:.2e}, smooth {err2:.2e}")
    assert err < 1e-4
    assert err2 < 5e-4


def test_split_bf16_steps_3d():
    m = inputs.tet_grid(3, seed=6, permute=True)
    d = oracle.Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, 4)
    op = oracle.Maxwell3D(d, 1.0)
    dt = cfl_dt(d, 4)
    q0 = oracle.cavity_mode_3d(d.x, d.y, d.z, 0.0)
    want = op.run(q0, dt, 30)
    with dgw.Solver(m, 4, prec="split_bf16") as s:
        s.set_fields(q0)
        s.advance_steps(30, dt)
        err = rel(s.get_fields(), want)
    print(f"3D split_bf16 30 steps vs oracle: {err:.2e}")
    assert err < 1e-4


def test_3d_split_bf16_full_size_vs_closed_form():
    """The 663552-tetrahedron cavity to t = 1 with the split-BF16 stage."""
    m = inputs.tet_grid(48, seed=5)
    with dgw.Solver(m, 4, prec="split_bf16") as s:
        s.set_cavity_mode(1, 1, 1)
        n = s.advance(1.0)
        err = s.cavity_error(1, 1, 1, 1.0)
        print(f"3D split_bf16 663552 tets to t=1 in {n} steps: rel L2 vs closed form {err:.2e}")
        assert err < 1e-4


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_wave_private_partition_3d(prec):
    """The wave-private work partition (no LDS sharing across waves, no
    work-group barriers) against the oracle: one right-hand side and ten
    steps on a permuted 3^3 x 6 mesh at order 4."""
    m = inputs.tet_grid(3, seed=9, permute=True)
    d = oracle.Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, 4)
    op = oracle.Maxwell3D(d, 1.0)
    dt = cfl_dt(d, 4)
    tol = 1e-5 if prec == "fp32" else 1e-4
    q = np.random.default_rng(9).standard_normal((6, d.K, d.Np))
    q0 = oracle.cavity_mode_3d(d.x, d.y, d.z, 0.0)
    with dgw.Solver(m, 4, prec=prec, wave_private=1) as s:
        assert s.info()["wave_private"] == 1
        err = rel(s.rhs(q), op.rhs(q))
        s.set_fields(q0)
        s.advance_steps(10, dt)
        err2 = rel(s.get_fields(), op.run(q0, dt, 10))
    print(f"3D wave-private {prec}: rhs {err:.2e}, 10 steps {err2:.2e}")
    assert err < tol and err2 < tol
