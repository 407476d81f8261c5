"""GPU parity of the fused 2D stage kernel (through the C ABI) against the
FP64 oracle, on the same seeded meshes and fields.

Tolerances: 1e-5 relative L2 for the fields after a run (the FP32 target),
1e-5 for a single right-hand side of random data (FP32 arithmetic on an
operator whose entries reach ~N^2/h; measured values are printed)."""

import math

import numpy as np
import pytest

import oracle
from oracle.maxwell import cfl_dt
from paper_1304_5546_amd import dgw, inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _setup(m, N, alpha=1.0, renumber=True):
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, N, eps=m.eps, mu=m.mu)
    op = oracle.Maxwell2D(d, alpha)
    s = dgw.Solver(m, N, alpha=alpha, renumber=renumber)
    return d, op, s


RHS_CASES = [
    # (grid s, order N, seed, permute, materials, alpha)
    (8, 3, 1, False, False, 1.0),     # the small cavity: 128 triangles, N = 3
    (20, 5, 2, True, False, 1.0),     # 800 elements: 13 tiles with a ragged tail
    (13, 7, 3, True, True, 1.0),      # disk inclusion eps = 2.25
    (6, 1, 4, False, False, 0.0),     # central flux
    (9, 8, 5, True, True, 0.5),       # highest order, blended flux
    (1, 2, 6, False, False, 1.0),     # 2 elements: every face but one on the wall
]


@pytest.mark.parametrize("s,N,seed,permute,mat,alpha", RHS_CASES)
def test_single_rhs_parity(s, N, seed, permute, mat, alpha):
    m = inputs.tri_grid(s, seed=seed, permute=permute)
    if mat:
        m.eps = inputs.disk_inclusion_eps(m, (0.1, -0.2), 0.45)
        m.mu = np.where(np.arange(m.K) % 3 == 0, 1.5, 1.0)
    d, op, sol = _setup(m, N, alpha)
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(sol.shape)
    want = op.rhs(q)
    got = sol.rhs(q)
    err = rel(got, want)
    print(f"rhs parity s={s} N={N} K={m.K}: rel L2 {err:.2e}")
    assert err < 1e-5
    # smooth data (the cavity mode): the same bound
    q = oracle.cavity_mode_2d(d.x, d.y, 0.3, 2, 1)
    err2 = rel(sol.rhs(q), op.rhs(q))
    print(f"   smooth: {err2:.2e}")
    assert err2 < 1e-5


def test_c1_cavity_100_steps_parity():
    """8x8 grid, 128 triangles, N=3, Ez0 = sin(pi x) sin(pi y), 100 steps at CFL dt."""
    m = inputs.tri_grid(8, seed=1)
    d, op, sol = _setup(m, 3)
    dt = cfl_dt(d, 3)
    assert abs(sol.cfl_dt() / dt - 1) < 1e-13
    q0 = oracle.cavity_mode_2d(d.x, d.y, 0.0, 1, 1)
    sol.set_fields(q0)
    sol.advance_steps(100, dt)
    got = sol.get_fields()
    want = op.run(q0, dt, 100)
    err = rel(got, want)
    print(f"C1 100 steps: GPU vs oracle {err:.2e}")
    assert err < 1e-5
    # closed-form error: same within the parity tolerance
    ex = oracle.cavity_mode_2d(d.x, d.y, 100 * dt, 1, 1)
    assert abs(op.rel_l2(got, ex) - op.rel_l2(want, ex)) < 1e-5
    # FP64 device reductions agree with the oracle on the GPU's own fields
    assert abs(sol.energy() / op.energy(got) - 1) < 1e-12
    e_dev = sol.cavity_error(1, 1, 0, 100 * dt)
    assert abs(e_dev / op.rel_l2(got, ex) - 1) < 1e-9


def test_material_run_parity_and_energy_decay():
    m = inputs.tri_grid(10, seed=7, permute=True)
    m.eps = inputs.disk_inclusion_eps(m, (0.2, 0.1), 0.4)
    d, op, sol = _setup(m, 5)
    dt = cfl_dt(d, 5)
    q0 = oracle.cavity_mode_2d(d.x, d.y, 0.0, 2, 3)
    sol.set_fields(q0)
    energies = [sol.energy()]
    for _ in range(6):
        sol.advance_steps(10, dt)
        energies.append(sol.energy())
    want = op.run(q0, dt, 60)
    err = rel(sol.get_fields(), want)
    print(f"material 60 steps: {err:.2e}")
    assert err < 1e-5
    # weighted energy (mu for H, eps for Ez) agrees with the oracle's and decays
    assert abs(energies[-1] / op.energy(sol.get_fields()) - 1) < 1e-12
    assert all(b <= a * (1 + 1e-6) for a, b in zip(energies, energies[1:]))


def test_renumbering_is_bitwise_invariant():
    m = inputs.tri_grid(16, seed=9, permute=True)
    res = []
    for ren in (True, False):
        with dgw.Solver(m, 4, renumber=ren) as s:
            s.set_cavity_mode(1, 2)
            s.advance_steps(20)
            res.append(s.get_fields())
    assert np.array_equal(res[0], res[1])


def test_set_get_and_device_init():
    m = inputs.tri_grid(11, seed=2, permute=True)
    d, op, sol = _setup(m, 6)
    rng = np.random.default_rng(3)
    q = rng.standard_normal(sol.shape)
    sol.set_fields(q)
    assert np.array_equal(sol.get_fields(), q.astype(np.float32).astype(np.float64))
    sol.set_cavity_mode(3, 2)
    ex = oracle.cavity_mode_2d(d.x, d.y, 0.0, 3, 2)
    assert np.abs(sol.get_fields() - ex).max() < 1e-7


def test_advance_to_t_final_counts_steps():
    m = inputs.tri_grid(6, seed=1)
    d, op, sol = _setup(m, 2)
    n = sol.advance(0.5)
    dt = cfl_dt(d, 2)
    assert n == math.ceil(0.5 / dt - 1e-12)
    info = sol.info()
    assert info["steps"] == n and abs(info["t"] - 0.5) < 1e-12 and info["solve_ms"] > 0


def test_device_pointer_path_matches_host_path():
    torch = pytest.importorskip("torch")
    m = inputs.tri_grid(12, seed=4, permute=True)
    N = 5
    stream = torch.cuda.Stream()
    with dgw.Solver(m, N, stream=stream) as s1, dgw.Solver(m, N) as s2:
        rng = np.random.default_rng(5)
        q = rng.standard_normal(s1.shape).astype(np.float32)
        qd = torch.from_numpy(q).cuda()
        s1.set_fields_dev(qd, stream)
        dt = s1.cfl_dt()
        s1.launch_steps(7, dt, stream)
        out = torch.empty_like(qd)
        s1.get_fields_dev(out, stream)
        stream.synchronize()
        s2.set_fields(q.astype(np.float64))
        s2.advance_steps(7, dt)
        assert np.array_equal(out.cpu().numpy().astype(np.float64), s2.get_fields())


def test_c2_full_size_one_step_parity():
    """Full 256x256 grid (131072 permuted triangles), N=5, mode (2,3): one
    LSRK4 step of the GPU against the oracle on the whole mesh, in the launch
    configuration the benchmark times."""
    m = inputs.tri_grid(256, seed=2, permute=True)
    d, op, sol = _setup(m, 5)
    dt = cfl_dt(d, 5)
    q0 = oracle.cavity_mode_2d(d.x, d.y, 0.0, 2, 3)
    sol.set_fields(q0)
    sol.advance_steps(1, dt)
    q = q0.copy()
    res = np.zeros_like(q)
    op.lsrk4_step(q, res, dt)
    got = sol.get_fields()
    err = rel(got, q)
    per_el = np.abs(got - q).max(axis=(0, 2)) / np.abs(q).max()
    print(f"C2 one step: rel L2 {err:.2e}, worst element {int(per_el.argmax())} max-abs {per_el.max():.2e}")
    assert err < 1e-6
    assert per_el.max() < 1e-5


def test_c2_full_length_vs_closed_form():
    """The full C2 solve to t = 1 at the CFL step: the GPU's FP32 result
    against the closed-form mode, whose distance from the FP64 discrete
    solution (N=5, h=2/256) is far below the 1e-5 budget."""
    m = inputs.tri_grid(256, seed=2, permute=True)
    with dgw.Solver(m, 5) as s:
        s.set_cavity_mode(2, 3)
        n = s.advance(1.0)
        err = s.cavity_error(2, 3, 0, 1.0)
        print(f"C2 to t=1 in {n} steps: rel L2 vs closed form {err:.2e}")
        assert err < 1e-5
