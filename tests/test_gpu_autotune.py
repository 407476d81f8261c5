"""Automated tuning over kernel variants and launch shapes (dgw_autotune):
the state is restored bitwise, the choice is the fastest candidate, and a
tuned solver computes bitwise what an untuned solver of the chosen kernel
computes (per-element arithmetic does not depend on the launch shape).
Different kernels may round differently, so the comparison is made from the
fields at the tuning point on.  Each tuned solve is also compared with the
FP64 oracle: random fields, tuning, then steps at the CFL step, against the
oracle's steps from the same fields (relative L2 within 1e-5 for FP32, 1e-4
for split-BF16, 1e-12 for FP64)."""

import numpy as np
import pytest

import oracle
from oracle.maxwell import cfl_dt
from paper_1304_5546_amd import dgw, inputs

ORACLE_TOL = {"fp32": 1e-5, "split_bf16": 1e-4, "fp64": 1e-12}


def _tuned_vs_oracle(m, N, steps, **kw):
    if m.dim == 2:
        d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, N)
        op = oracle.Maxwell2D(d)
    else:
        d = oracle.Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, N)
        op = oracle.Maxwell3D(d)
    dt = cfl_dt(d, N)
    q = np.random.default_rng(11).standard_normal((3 if m.dim == 2 else 6, d.K, d.Np)) * 0.1
    want = op.run(q, dt, steps)
    with dgw.Solver(m, N, **kw) as s:
        s.set_fields(q)
        t = s.autotune(stages=5)
        s.advance_steps(steps, dt)
        got = s.get_fields()
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    print(f"tuned {kw} (kernel {t['kernel']} x{t['groups_per_cu']}) vs oracle after {steps} steps: {err:.2e}")
    assert err < ORACLE_TOL[kw.get("prec", "fp32")]

pytestmark = pytest.mark.gpu


def _check_tuned(m, N, steps, **kw):
    with dgw.Solver(m, N, **kw) as s:
        rng = np.random.default_rng(1)
        q = rng.standard_normal(s.shape) * 0.1
        s.set_fields(q)
        s.advance_steps(3)  # a nonzero residual to preserve
        before, e_before = s.get_fields(), s.energy()
        t = s.autotune(stages=5)
        print(f"autotune {kw}: choice kernel {t['kernel']} x{t['groups_per_cu']} "
              f"{t['best_us']:.2f} us; tried {[(c['kernel'], c['groups_per_cu'], round(c['us'], 2)) for c in t['tried']]}")
        assert np.array_equal(s.get_fields(), before)
        assert s.energy() == e_before
        assert t["best_us"] == min(c["us"] for c in t["tried"])
        assert (t["kernel"], t["groups_per_cu"]) in [(c["kernel"], c["groups_per_cu"]) for c in t["tried"]]
        s.advance_steps(steps)
        tuned = s.get_fields()
    # the same steps, untuned, on the chosen kernel (default launch shape),
    # from the fields the tuned solver had before tuning (a step starts with
    # RK coefficient a = 0, so the residual left by the previous step does not
    # enter it)
    kw2 = dict(kw)
    if m.dim == 2 and kw.get("prec", "fp32") in ("fp32", "fp64"):
        kw2["kernel"] = t["kernel"]
        if t["lane_elems"] == 2:
            kw2["lane_elems"] = 2
    if m.dim == 3:
        kw2["wave_private"] = t["wave_private"]
    with dgw.Solver(m, N, **kw2) as s:
        s.set_fields(before)
        s.advance_steps(steps)
        plain = s.get_fields()
    assert np.array_equal(tuned, plain), "tuned and untuned solves differ"
    return t


def test_autotune_fp32_2d():
    m = inputs.tri_grid(48, seed=3, permute=True)
    t = _check_tuned(m, 5, 10)
    kernels = {c["kernel"] for c in t["tried"]}
    assert kernels == {1, 2, 3, 4}
    # the derivative-first kernel with one and with two elements per lane
    assert {c["lane_elems"] for c in t["tried"] if c["kernel"] == 3} == {1, 2}
    _tuned_vs_oracle(m, 5, 10)


def test_autotune_fp64_2d():
    m = inputs.tri_grid(32, seed=4, permute=True)
    t = _check_tuned(m, 4, 10, prec="fp64")
    assert {c["kernel"] for c in t["tried"]} == {1, 3}
    _tuned_vs_oracle(m, 4, 10, prec="fp64")


def test_autotune_split_and_3d_vary_the_launch_shape_only():
    m = inputs.tri_grid(40, seed=5)
    t = _check_tuned(m, 5, 6, prec="split_bf16")
    assert len({c["kernel"] for c in t["tried"]}) == 1
    _tuned_vs_oracle(m, 5, 6, prec="split_bf16")
    m3 = inputs.tet_grid(6, seed=2)
    t = _check_tuned(m3, 3, 4)
    assert len({c["kernel"] for c in t["tried"]}) == 1
    # the shared pair window and the wave-private partition
    assert {c["wave_private"] for c in t["tried"]} == {0, 1}
    _tuned_vs_oracle(m3, 3, 4)
