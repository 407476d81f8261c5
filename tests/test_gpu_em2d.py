"""GPU parity of the element-major 2D FP32 stage kernel (kernel 4: fields
stored element by element, derivative operator packed by output slot, LDS
windows of four tiles) against the FP64 oracle, through the C ABI.  FP32
bounds as for the other FP32 kernels: 1e-5 relative L2 per right-hand side
and over multi-step runs; at the full 512 x 512 size one LSRK4 step and one
right-hand side with the per-element max-abs error beside the L2."""

import numpy as np
import pytest

import oracle
from oracle.maxwell import cfl_dt
from paper_1304_5546_amd import dgw, inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def compare(got, want, label):
    l2 = rel(got, want)
    per_el = np.abs(got - want).max(axis=(0, 2))
    k = int(np.argmax(per_el))
    emax = float(per_el[k] / np.abs(want).max())
    print(f"{label}: rel L2 {l2:.2e}, worst element {k} max-abs {emax:.2e}", flush=True)
    return l2, emax


CASES = [
    # (grid s, order N, seed, permute, materials, alpha)
    (8, 3, 1, False, False, 1.0),
    (20, 5, 2, True, False, 1.0),     # 13 tiles: three windows, the last one ragged
    (13, 7, 3, True, True, 1.0),
    (6, 1, 4, False, False, 0.0),     # central flux
    (9, 8, 5, True, True, 0.5),       # order 8: windows of two tiles
    (1, 2, 6, False, False, 1.0),     # 2 elements
    (11, 4, 7, True, False, 1.0),
    (10, 6, 8, True, True, 1.0),
    (40, 7, 9, True, False, 1.0),     # 3200 elements: 13 windows of 4 tiles
]


def _mesh(s, seed, permute, mat):
    m = inputs.tri_grid(s, seed=seed, permute=permute)
    if mat:
        m.eps = inputs.disk_inclusion_eps(m, (0.1, -0.2), 0.45)
        m.mu = np.where(np.arange(m.K) % 3 == 0, 1.5, 1.0)
    return m


@pytest.mark.parametrize("s,N,seed,permute,mat,alpha", CASES)
def test_em2d_rhs_parity(s, N, seed, permute, mat, alpha):
    m = _mesh(s, seed, permute, mat)
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, N, eps=m.eps, mu=m.mu)
    op = oracle.Maxwell2D(d, alpha)
    with dgw.Solver(m, N, alpha=alpha, kernel=4) as sol:
        assert sol.info()["kernel"] == 4
        rng = np.random.default_rng(seed)
        q = rng.standard_normal(sol.shape)
        err = rel(sol.rhs(q), op.rhs(q))
        qs = oracle.cavity_mode_2d(d.x, d.y, 0.3, 2, 1)
        err2 = rel(sol.rhs(qs), op.rhs(qs))
    print(f"kernel 4 rhs s={s} N={N} K={m.K}: random {err:.2e}, smooth {err2:.2e}")
    assert err < 1e-5
    assert err2 < 1e-5


def test_em2d_c1_100_steps_material_run_and_reductions():
    m = inputs.tri_grid(8, seed=1)
    d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, 3)
    op = oracle.Maxwell2D(d)
    dt = cfl_dt(d, 3)
    q0 = oracle.cavity_mode_2d(d.x, d.y, 0.0, 1, 1)
    want = op.run(q0, dt, 100)
    with dgw.Solver(m, 3, kernel=4) as sol:
        sol.set_fields(q0)
        e0 = sol.energy()
        sol.advance_steps(100, dt)
        got = sol.get_fields()
        err = rel(got, want)
        assert abs(sol.energy() / op.energy(got) - 1) < 1e-12
        assert sol.energy() < e0
        # device initialisation of the mode in the element-major layout
        sol.set_cavity_mode(1, 1)
        assert np.abs(sol.get_fields() - q0).max() < 1e-7
    print(f"kernel 4 C1 100 steps: {err:.2e}")
    assert err < 1e-5
    mm = _mesh(12, 3, True, True)
    dm = oracle.Discretization2D(mm.vx, mm.vy, mm.elem_verts, 5, eps=mm.eps, mu=mm.mu)
    opm = oracle.Maxwell2D(dm)
    dtm = cfl_dt(dm, 5)
    qm = oracle.cavity_mode_2d(dm.x, dm.y, 0.0, 1, 2)
    wantm = opm.run(qm, dtm, 60)
    with dgw.Solver(mm, 5, kernel=4) as sol:
        sol.set_fields(qm)
        sol.advance_steps(60, dtm)
        errm = rel(sol.get_fields(), wantm)
    print(f"kernel 4 material 60 steps: {errm:.2e}")
    assert errm < 1e-5


def test_em2d_device_fields_roundtrip():
    import torch

    m = inputs.tri_grid(10, seed=4, permute=True)
    with dgw.Solver(m, 6, kernel=4) as sol:
        q = np.random.default_rng(4).standard_normal(sol.shape).astype(np.float32)
        qt = torch.from_numpy(q).cuda()
        sol.set_fields_dev(qt)
        back = torch.empty_like(qt)
        sol.get_fields_dev(back)
        torch.cuda.synchronize()
        assert np.array_equal(back.cpu().numpy(), q)
        assert np.array_equal(sol.get_fields().astype(np.float32), q)


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
    qr = np.random.default_rng(3).standard_normal(q0.shape)
    return dict(m=m, dt=dt, q0=q0, q1=q1, qr=qr, rhs=op.rhs(qr))


def test_em2d_c3_full_size_one_step_and_rhs(c3):
    with dgw.Solver(c3["m"], 7, kernel=4) as s:
        s.set_fields(c3["q0"])
        s.advance_steps(1, c3["dt"])
        l2, emax = compare(s.get_fields(), c3["q1"], "C3 kernel 4 one step")
        assert l2 < 1e-6 and emax < 1e-5
        l2, emax = compare(s.rhs(c3["qr"]), c3["rhs"], "C3 kernel 4 rhs of random data")
        assert l2 < 1e-5 and emax < 1e-4


def test_em2d_c3_to_t1_vs_closed_form():
    m = inputs.tri_grid(512, seed=3)
    with dgw.Solver(m, 7, kernel=4) as s:
        s.set_cavity_mode(2, 3)
        n = s.advance(1.0)
        err = s.cavity_error(2, 3, 0, 1.0)
    print(f"C3 kernel 4 to t=1 in {n} steps: rel L2 vs closed form {err:.2e}")
    assert err < 1e-5
