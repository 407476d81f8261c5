"""Pins of the oracle's diagnostics -- the discrete energy and the relative
L2 error in the mass-matrix norm -- against values the mathematics fixes
(CPU only).

  * Polynomial fields of degree <= N are reproduced exactly by the nodal
    basis, and J_k u^T M u is then the exact integral of u^2 over element k.
    On the jittered meshes the domain is exactly [-1,1]^2 (or [-1,1]^3:
    boundary vertices are not moved), so the integrals of x^2, x^2 y^2, ...
    over the whole domain are known in closed form.
  * Fields constant on each element integrate to (element area) * value^2;
    areas and volumes are computed here from the vertex coordinates
    (shoelace / triple product), not from the oracle's Jacobians.
  * The closed-form cavity mode carries the energy eps/2 at every time
    (its electric and magnetic parts trade places), which the interpolated
    mode reproduces to the interpolation error.

Each pin is also run against an oracle with a planted mistake (swapped
eps/mu weights, a dropped 1/2, a missing square root, Jacobians left out),
which must fail it.
"""

import math

import numpy as np
import pytest

from oracle import Discretization2D, Discretization3D, Maxwell2D, Maxwell3D, cavity_mode_2d
from paper_1304_5546_amd import inputs


def _graded(m):
    """Move the vertices by x -> x + 0.4 sin(pi x) / pi (and the same in y):
    a monotone map of [-1,1] onto itself, so the domain stays the square
    while element areas vary by a factor of about five."""
    g = lambda v: v + 0.4 * np.sin(np.pi * v) / np.pi
    m.vx, m.vy = g(m.vx), g(m.vy)
    return m


def _areas(m):
    P = [np.stack([m.vx[m.elem_verts[:, i]], m.vy[m.elem_verts[:, i]]], 1) for i in range(3)]
    a, b = P[1] - P[0], P[2] - P[0]
    return 0.5 * (a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0])


def _volumes(m):
    P = [np.stack([m.vx[m.elem_verts[:, i]], m.vy[m.elem_verts[:, i]], m.vz[m.elem_verts[:, i]]], 1)
         for i in range(4)]
    return np.einsum("ij,ij->i", P[1] - P[0], np.cross(P[2] - P[0], P[3] - P[0])) / 6.0


# ---------------------------------------------------------------- planted mistakes (the oracle with one error)

class _SwappedWeights(Maxwell2D):
    def energy(self, q):
        d = self.d
        flipped = Maxwell2D.__new__(Maxwell2D)
        flipped.d = type("D", (), {})()
        flipped.d.__dict__.update(d.__dict__)
        flipped.d.eps, flipped.d.mu = d.mu, d.eps
        return Maxwell2D.energy(flipped, q)


class _NoHalf(Maxwell2D):
    def energy(self, q):
        return 2.0 * super().energy(q)


class _NoJacobian(Maxwell2D):
    def energy(self, q):
        d = self.d
        J = d.J
        d.J = np.ones_like(J)
        try:
            return super().energy(q)
        finally:
            d.J = J


class _NoSqrt(Maxwell2D):
    def rel_l2(self, q, ref):
        return super().rel_l2(q, ref) ** 2


class _NoJacobianL2(Maxwell2D):
    def rel_l2(self, q, ref):
        d = self.d
        J = d.J
        d.J = np.ones_like(J)
        try:
            return super().rel_l2(q, ref)
        finally:
            d.J = J


# ---------------------------------------------------------------- the pins as functions of an operator

def _energy_polynomial_error(cls, N=3):
    """Hx = x, Hy = y, Ez = x y with uniform eps = 2.25, mu = 0.7:
    E = 1/2 (mu (4/3 + 4/3) + eps 4/9) over [-1,1]^2."""
    m = _graded(inputs.tri_grid(5, seed=31))
    eps, mu = 2.25, 0.7
    d = Discretization2D(m.vx, m.vy, m.elem_verts, N, eps=np.full(m.K, eps), mu=np.full(m.K, mu))
    op = cls(d)
    q = np.stack([d.x, d.y, d.x * d.y])
    exact = 0.5 * (mu * 8.0 / 3.0 + eps * 4.0 / 9.0)
    return abs(op.energy(q) / exact - 1.0)


def _energy_piecewise_error(cls, N=2):
    """Per-element constants a, b, c and random per-element eps, mu:
    E = 1/2 sum_k area_k (mu_k (a_k^2 + b_k^2) + eps_k c_k^2)."""
    m = _graded(inputs.tri_grid(6, seed=32, permute=True))
    rng = np.random.default_rng(3)
    eps = rng.uniform(1.0, 4.0, m.K)
    mu = rng.uniform(0.5, 2.0, m.K)
    abc = rng.standard_normal((3, m.K))
    d = Discretization2D(m.vx, m.vy, m.elem_verts, N, eps=eps, mu=mu)
    op = cls(d)
    q = np.repeat(abc[:, :, None], d.Np, axis=2)
    exact = 0.5 * float(np.sum(_areas(m) * (mu * (abc[0] ** 2 + abc[1] ** 2) + eps * abc[2] ** 2)))
    return abs(op.energy(q) / exact - 1.0)


def _energy_cavity_error(cls):
    """The closed-form mode (2,1) with uniform eps = 2, mu = 0.5 at t = 0.13
    (both parts non-zero): energy eps/2 = 1."""
    m = inputs.tri_grid(24, seed=33)
    eps, mu = 2.0, 0.5
    d = Discretization2D(m.vx, m.vy, m.elem_verts, 6, eps=np.full(m.K, eps), mu=np.full(m.K, mu))
    op = cls(d)
    q = cavity_mode_2d(d.x, d.y, 0.13, 2, 1, eps=eps, mu=mu)
    return abs(op.energy(q) / (0.5 * eps) - 1.0)


def _rel_l2_polynomial_error(cls, N=4):
    """ref = (x, 0, 0), q = ref + (0, 0, x y): sqrt((4/9) / (4/3)) = 1/sqrt(3);
    q = c ref: |c - 1|."""
    m = _graded(inputs.tri_grid(5, seed=34))
    d = Discretization2D(m.vx, m.vy, m.elem_verts, N)
    op = cls(d)
    z = np.zeros_like(d.x)
    ref = np.stack([d.x, z, z])
    q = np.stack([d.x, z, d.x * d.y])
    e1 = abs(op.rel_l2(q, ref) - 1.0 / math.sqrt(3.0))
    e2 = abs(op.rel_l2(-0.5 * ref, ref) - 1.5)
    return max(e1, e2)


def _rel_l2_piecewise_error(cls, N=2):
    """Per-element constants on a jittered mesh:
    sqrt(sum_k area_k |q_k - r_k|^2 / sum_k area_k |r_k|^2)."""
    m = _graded(inputs.tri_grid(7, seed=35, permute=True))
    rng = np.random.default_rng(4)
    qc = rng.standard_normal((3, m.K))
    rc = rng.standard_normal((3, m.K))
    d = Discretization2D(m.vx, m.vy, m.elem_verts, N)
    op = cls(d)
    q = np.repeat(qc[:, :, None], d.Np, axis=2)
    r = np.repeat(rc[:, :, None], d.Np, axis=2)
    A = _areas(m)
    exact = math.sqrt(float(np.sum(A * ((qc - rc) ** 2).sum(0)) / np.sum(A * (rc ** 2).sum(0))))
    return abs(op.rel_l2(q, r) / exact - 1.0)


# ---------------------------------------------------------------- tests

def test_energy_of_polynomial_fields_is_exact():
    assert _energy_polynomial_error(Maxwell2D) < 1e-13


def test_energy_of_piecewise_constant_fields_with_random_materials():
    assert _energy_piecewise_error(Maxwell2D) < 1e-13


def test_energy_of_cavity_mode_is_half_eps():
    err = _energy_cavity_error(Maxwell2D)
    print(f"cavity energy relative error {err:.2e}")
    assert err < 1e-7


def test_rel_l2_of_polynomial_fields_is_exact():
    assert _rel_l2_polynomial_error(Maxwell2D) < 1e-13


def test_rel_l2_of_piecewise_constant_fields_on_jittered_mesh():
    assert _rel_l2_piecewise_error(Maxwell2D) < 1e-13


@pytest.mark.parametrize("cls", [_SwappedWeights, _NoHalf, _NoJacobian])
def test_planted_energy_mistakes_fail_a_pin(cls):
    errs = [_energy_polynomial_error(cls), _energy_piecewise_error(cls), _energy_cavity_error(cls)]
    assert max(errs) > 1e-3, errs


@pytest.mark.parametrize("cls", [_NoSqrt, _NoJacobianL2])
def test_planted_rel_l2_mistakes_fail_a_pin(cls):
    errs = [_rel_l2_polynomial_error(cls), _rel_l2_piecewise_error(cls)]
    assert max(errs) > 1e-3, errs


def test_energy_and_rel_l2_3d():
    """3D: polynomial fields (x, y, z, x y, y z, 1) have energy
    1/2 (3 * 8/3 + 2 * 8/9 + 8); per-element constants give
    1/2 sum_k vol_k |c_k|^2; rel_l2 of (x,0,..) + (0,..,x y z) against
    (x,0,..) is sqrt((8/27) / (8/3)) = 1/3."""
    m = inputs.tet_grid(3, seed=36)
    d = Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, 3)
    op = Maxwell3D(d)
    x, y, z = d.x, d.y, d.z
    q = np.stack([x, y, z, x * y, y * z, np.ones_like(x)])
    exact = 0.5 * (3 * 8.0 / 3.0 + 2 * 8.0 / 9.0 + 8.0)
    assert abs(op.energy(q) / exact - 1) < 1e-13
    rng = np.random.default_rng(5)
    c = rng.standard_normal((6, m.K))
    qc = np.repeat(c[:, :, None], d.Np, axis=2)
    exact = 0.5 * float(np.sum(_volumes(m) * (c ** 2).sum(0)))
    assert abs(op.energy(qc) / exact - 1) < 1e-13
    zero = np.zeros_like(x)
    ref = np.stack([x, zero, zero, zero, zero, zero])
    qq = np.stack([x, zero, zero, zero, zero, x * y * z])
    assert abs(op.rel_l2(qq, ref) - 1.0 / 3.0) < 1e-13
