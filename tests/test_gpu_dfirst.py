"""GPU parity of the derivative-first FP32 2D stage kernel (kernel 3) against
the FP64 oracle and against the fused-operand MFMA kernel (kernel 2), through
the C ABI.  FP32 bounds as for the other FP32 kernels: 1e-5 relative L2."""

import numpy as np
import pytest

import oracle
from oracle.maxwell import cfl_dt
from paper_1304_5546_amd import dgw, inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


CASES = [
    # (grid s, order N, seed, permute, materials, alpha)
    (8, 3, 1, False, False, 1.0),
    (20, 5, 2, True, False, 1.0),     # 13 tiles, ragged tail
    (13, 7, 3, True, True, 1.0),
    (6, 1, 4, False, False, 0.0),     # central flux
    (9, 8, 5, True, True, 0.5),
    (1, 2, 6, False, False, 1.0),     # 2 elements
    (11, 4, 7, True, False, 1.0),
    (10, 6, 8, True, True, 1.0),
]


def _mesh(s, seed, permute, mat):
    m = inputs.tri_grid(s, seed=seed, permute=permute)
    if mat:
        m.eps = inputs.disk_inclusion_eps(m, (0.1, -0.2), 0.45)
        m.mu = np.where(np.arange(m.K) % 3 == 0, 1.5, 1.0)
    return m


@pytest.mark.parametrize("lane_elems", [1, 2])
@pytest.mark.parametrize("s,N,seed,permute,mat,alpha", CASES)
def test_dfirst_rhs_parity(s, N, seed, permute, mat, alpha, lane_elems):
    """One and two elements per lane (the work partitions dgw_autotune
    searches) against the oracle."""
    m = _mesh(s, seed, permute, mat)
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, N, eps=m.eps, mu=m.mu)
    op = oracle.Maxwell2D(d, alpha)
    with dgw.Solver(m, N, alpha=alpha, kernel=3, lane_elems=lane_elems) as sol:
        assert sol.info()["lane_elems"] == lane_elems
        rng = np.random.default_rng(seed)
        q = rng.standard_normal(sol.shape)
        err = rel(sol.rhs(q), op.rhs(q))
        qs = oracle.cavity_mode_2d(d.x, d.y, 0.3, 2, 1)
        err2 = rel(sol.rhs(qs), op.rhs(qs))
    print(f"kernel 3 x{lane_elems} rhs s={s} N={N} K={m.K}: random {err:.2e}, smooth {err2:.2e}")
    assert err < 1e-5
    assert err2 < 1e-5


def test_dfirst_c1_100_steps_and_material_run():
    m = inputs.tri_grid(8, seed=1)
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, 3)
    op = oracle.Maxwell2D(d)
    dt = cfl_dt(d, 3)
    q0 = oracle.cavity_mode_2d(d.x, d.y, 0.0, 1, 1)
    with dgw.Solver(m, 3, kernel=3) as sol:
        sol.set_fields(q0)
        sol.advance_steps(100, dt)
        err = rel(sol.get_fields(), op.run(q0, dt, 100))
    print(f"kernel 3 C1 100 steps: {err:.2e}")
    assert err < 1e-5
    m = inputs.tri_grid(10, seed=7, permute=True)
    m.eps = inputs.disk_inclusion_eps(m, (0.2, 0.1), 0.4)
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, 5, eps=m.eps, mu=m.mu)
    op = oracle.Maxwell2D(d)
    dt = cfl_dt(d, 5)
    q0 = oracle.cavity_mode_2d(d.x, d.y, 0.0, 2, 3)
    with dgw.Solver(m, 5, kernel=3) as sol:
        sol.set_fields(q0)
        e0 = sol.energy()
        sol.advance_steps(60, dt)
        err = rel(sol.get_fields(), op.run(q0, dt, 60))
        assert sol.energy() <= e0 * (1 + 1e-6)
    print(f"kernel 3 material 60 steps: {err:.2e}")
    assert err < 1e-5


def test_dfirst_matches_fused_operand_kernel():
    m = inputs.tri_grid(24, seed=9, permute=True)
    out = []
    for kernel in (2, 3):
        with dgw.Solver(m, 7, kernel=kernel) as sol:
            sol.set_cavity_mode(2, 1)
            sol.advance_steps(50)
            out.append(sol.get_fields())
    err = rel(out[1], out[0])
    print(f"kernel 3 vs kernel 2 after 50 steps: {err:.2e}")
    assert err < 1e-5


def test_dfirst_c2_full_size():
    """Full 256x256 grid (131072 permuted triangles), N=5, mode (2,3): one
    step against the oracle on the whole mesh, then to t = 1 against the
    closed form, in the launch configuration the benchmark times."""
    m = inputs.tri_grid(256, seed=2, permute=True)
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, 5)
    op = oracle.Maxwell2D(d)
    dt = cfl_dt(d, 5)
    q0 = oracle.cavity_mode_2d(d.x, d.y, 0.0, 2, 3)
    with dgw.Solver(m, 5, kernel=3) as sol:
        sol.set_fields(q0)
        sol.advance_steps(1, dt)
        got = sol.get_fields()
        sol.set_cavity_mode(2, 3)
        n = sol.advance(1.0)
        e1 = sol.cavity_error(2, 3, 0, 1.0)
    q = q0.copy()
    res = np.zeros_like(q)
    op.lsrk4_step(q, res, dt)
    err = rel(got, q)
    print(f"kernel 3 C2 one step: {err:.2e}; to t=1 in {n} steps: {e1:.2e} vs closed form")
    assert err < 1e-6
    assert e1 < 1e-5
