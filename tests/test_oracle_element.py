"""Pins of the oracle's reference elements and geometry against closed forms,
symmetries, exact integration and the divergence theorem (CPU only)."""

import itertools
import math

import numpy as np
import pytest
from scipy import special

from oracle import Discretization2D, Discretization3D, RefElement2D, RefElement3D, lgl_nodes
from oracle.element import ALPHA_OPT_3D, nodes_2d, nodes_3d
from paper_1304_5546_amd import inputs


# ---------------------------------------------------------------- 1D nodes

def test_lgl_nodes_closed_forms():
    # Gauss-Lobatto-Legendre points: endpoints plus zeros of P_N'
    assert np.allclose(lgl_nodes(2), [-1, 0, 1], atol=1e-15)
    a = 1 / math.sqrt(5)
    assert np.allclose(lgl_nodes(3), [-1, -a, a, 1], atol=1e-15)
    b = math.sqrt(3 / 7)
    assert np.allclose(lgl_nodes(4), [-1, -b, 0, b, 1], atol=1e-15)
    c1 = math.sqrt(1 / 3 - 2 * math.sqrt(7) / 21)
    c2 = math.sqrt(1 / 3 + 2 * math.sqrt(7) / 21)
    assert np.allclose(lgl_nodes(5), [-1, -c2, -c1, c1, c2, 1], atol=1e-14)


@pytest.mark.parametrize("N", range(1, 9))
def test_lgl_quadrature_exact(N):
    # LGL quadrature with N+1 points is exact to degree 2N-1
    x = lgl_nodes(N)
    V = np.vander(x, N + 1, increasing=True)
    # weights from exactness on 1..x^N
    mom = np.array([(1 - (-1) ** (k + 1)) / (k + 1) for k in range(N + 1)])
    w = np.linalg.solve(V.T, mom)
    for k in range(2 * N):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-12


# ---------------------------------------------------------------- node sets

def _as_set(pts, decimals=10):
    return sorted(tuple(np.round(p, decimals)) for p in pts)


def test_nodes_2d_low_orders():
    r, s = nodes_2d(1)
    assert _as_set(np.c_[r, s]) == _as_set([[-1, -1], [1, -1], [-1, 1]])
    r, s = nodes_2d(2)
    assert _as_set(np.c_[r, s]) == _as_set([[-1, -1], [0, -1], [1, -1], [-1, 0], [0, 0], [-1, 1]])
    r, s = nodes_2d(3)
    inner = (np.abs(s + 1) > 1e-9) & (np.abs(r + 1) > 1e-9) & (np.abs(r + s) > 1e-9)
    assert inner.sum() == 1
    assert np.allclose([r[inner][0], s[inner][0]], [-1 / 3, -1 / 3], atol=1e-14)


@pytest.mark.parametrize("N", range(1, 9))
def test_nodes_2d_edges_are_lgl_and_symmetric(N):
    r, s = nodes_2d(N)
    x = lgl_nodes(N)
    assert np.allclose(np.sort(r[np.abs(s + 1) < 1e-10]), x, atol=1e-13)
    assert np.allclose(np.sort(s[np.abs(r + 1) < 1e-10]), x, atol=1e-13)
    assert np.allclose(np.sort(r[np.abs(r + s) < 1e-10]), x, atol=1e-13)
    # invariance of the node set under the triangle's symmetry group
    l1, l2, l3 = -(r + s) / 2, (1 + r) / 2, (1 + s) / 2
    base = _as_set(np.c_[r, s])
    for perm in itertools.permutations((l1, l2, l3)):
        rr = 2 * perm[1] - 1
        ss = 2 * perm[2] - 1
        assert _as_set(np.c_[rr, ss]) == base
    # all inside the triangle, distinct
    assert np.all(r >= -1 - 1e-12) and np.all(s >= -1 - 1e-12) and np.all(r + s <= 1e-12)
    assert len(base) == (N + 1) * (N + 2) // 2


@pytest.mark.parametrize("N", range(1, 7))
def test_nodes_3d_faces_are_2d_nodes(N):
    r, s, t = nodes_3d(N)
    # each face carries the 2D construction with the 3D blend parameter
    r2, s2 = nodes_2d(N, alpha=ALPHA_OPT_3D[N])
    tri = _as_set(np.c_[r2, s2])
    on = np.abs(t + 1) < 1e-10
    assert _as_set(np.c_[r[on], s[on]]) == tri
    on = np.abs(s + 1) < 1e-10
    assert _as_set(np.c_[r[on], t[on]]) == tri
    on = np.abs(r + 1) < 1e-10
    assert _as_set(np.c_[s[on], t[on]]) == tri
    on = np.abs(r + s + t + 1) < 1e-10
    assert _as_set(np.c_[s[on], t[on]]) == tri
    # symmetric under all permutations of the barycentric coordinates
    lam = np.c_[-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2]
    base = _as_set(np.c_[r, s, t])
    for perm in itertools.permutations(range(4)):
        L = lam[:, perm]
        assert _as_set(np.c_[2 * L[:, 1] - 1, 2 * L[:, 2] - 1, 2 * L[:, 3] - 1]) == base


# ---------------------------------------------------------------- exactness

def _single_triangle(seed):
    rng = np.random.default_rng(seed)
    P = np.array([[0.0, 0.0], [1.0, 0.1], [0.2, 0.9]]) + 0.2 * rng.standard_normal((3, 2))
    if (P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]) < 0:
        P = P[[0, 2, 1]]
    return P[:, 0], P[:, 1], np.array([[0, 1, 2]])


def _single_tet(seed):
    rng = np.random.default_rng(seed)
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]]) + 0.15 * rng.standard_normal((4, 3))
    if np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], 1)) < 0:
        P = P[[0, 2, 1, 3]]
    return P[:, 0], P[:, 1], P[:, 2], np.array([[0, 1, 2, 3]])


@pytest.mark.parametrize("N", range(1, 9))
def test_differentiation_exact_2d(N):
    vx, vy, ev = _single_triangle(N)
    d = Discretization2D(vx, vy, ev, N)
    x, y = d.x[0], d.y[0]
    ref = d.ref
    h = max(np.ptp(vx), np.ptp(vy))
    Dx = d.rx[0] * ref.Dr + d.sx[0] * ref.Ds
    Dy = d.ry[0] * ref.Dr + d.sy[0] * ref.Ds
    worst = 0.0
    for a in range(N + 1):
        for b in range(N + 1 - a):
            p = x ** a * y ** b
            px = a * x ** max(a - 1, 0) * y ** b if a else 0 * x
            py = b * x ** a * y ** max(b - 1, 0) if b else 0 * x
            worst = max(worst, np.abs(Dx @ p - px).max(), np.abs(Dy @ p - py).max())
    assert worst < 1e-11 * N * N / h
    # the test has teeth: degree N+1 is not differentiated exactly
    p = x ** (N + 1)
    assert np.abs(Dx @ p - (N + 1) * x ** N).max() > 1e-6


@pytest.mark.parametrize("N", range(1, 6))
def test_differentiation_exact_3d(N):
    vx, vy, vz, ev = _single_tet(N)
    d = Discretization3D(vx, vy, vz, ev, N)
    x, y, z = d.x[0], d.y[0], d.z[0]
    ref = d.ref
    D = [d.rx[0] * ref.Dr + d.sx[0] * ref.Ds + d.tx[0] * ref.Dt,
         d.ry[0] * ref.Dr + d.sy[0] * ref.Ds + d.ty[0] * ref.Dt,
         d.rz[0] * ref.Dr + d.sz[0] * ref.Ds + d.tz[0] * ref.Dt]
    worst = 0.0
    for a in range(N + 1):
        for b in range(N + 1 - a):
            for c in range(N + 1 - a - b):
                p = x ** a * y ** b * z ** c
                g = [a * x ** max(a - 1, 0) * y ** b * z ** c,
                     b * x ** a * y ** max(b - 1, 0) * z ** c,
                     c * x ** a * y ** b * z ** max(c - 1, 0)]
                for i in range(3):
                    worst = max(worst, np.abs(D[i] @ p - g[i]).max())
    assert worst < 1e-10 * N * N
    p = z ** (N + 1)
    assert np.abs(D[2] @ p - (N + 1) * z ** N).max() > 1e-6


# ---------------------------------------------------------------- quadrature helpers (independent of the oracle)

def _tri_quadrature(deg):
    """Collapsed (Duffy) Gauss rule on the reference triangle, exact to `deg`."""
    n = deg // 2 + 2
    xa, wa = special.roots_legendre(n)
    xb, wb = special.roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(xa, xb, indexing="ij")
    W = np.outer(wa, wb) * 0.5
    r = (1 + A) * (1 - B) / 2 - 1
    s = B
    return r.ravel(), s.ravel(), W.ravel()


def _tet_quadrature(deg):
    n = deg // 2 + 2
    xa, wa = special.roots_legendre(n)
    xb, wb = special.roots_jacobi(n, 1.0, 0.0)
    xc, wc = special.roots_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(xa, xb, xc, indexing="ij")
    W = wa[:, None, None] * wb[None, :, None] * wc[None, None, :] * 0.125
    r = (1 + A) * (1 - B) * (1 - C) / 4 - 1
    s = (1 + B) * (1 - C) / 2 - 1
    t = C
    return r.ravel(), s.ravel(), t.ravel(), W.ravel()


def test_quadrature_helpers_integrate_known_values():
    r, s, w = _tri_quadrature(6)
    assert abs(w.sum() - 2.0) < 1e-14
    # integral of (1+r) over the triangle = 4/3
    assert abs(np.dot(w, 1 + r) - 4 / 3) < 1e-14
    r, s, t, w = _tet_quadrature(6)
    assert abs(w.sum() - 4 / 3) < 1e-14
    assert abs(np.dot(w, (1 + r)) - 2 / 3) < 1e-14  # volume 4/3 times 1 + (centroid r = -1/2)


@pytest.mark.parametrize("N", [1, 3, 5, 8])
def test_mass_matrix_integrates_products_2d(N):
    ref = RefElement2D(N)
    qr, qs, qw = _tri_quadrature(2 * N)
    mons = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
    rng = np.random.default_rng(N)
    for _ in range(6):
        (a1, b1), (a2, b2) = (mons[i] for i in rng.integers(0, len(mons), 2))
        u, v = ref.r ** a1 * ref.s ** b1, ref.r ** a2 * ref.s ** b2
        exact = np.dot(qw, qr ** (a1 + a2) * qs ** (b1 + b2))
        assert abs(u @ ref.M @ v - exact) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 4])
def test_mass_matrix_integrates_products_3d(N):
    ref = RefElement3D(N)
    qr, qs, qt, qw = _tet_quadrature(2 * N)
    mons = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]
    rng = np.random.default_rng(N)
    for _ in range(6):
        m1, m2 = (mons[i] for i in rng.integers(0, len(mons), 2))
        u = ref.r ** m1[0] * ref.s ** m1[1] * ref.t ** m1[2]
        v = ref.r ** m2[0] * ref.s ** m2[1] * ref.t ** m2[2]
        exact = np.dot(qw, qr ** (m1[0] + m2[0]) * qs ** (m1[1] + m2[1]) * qt ** (m1[2] + m2[2]))
        assert abs(u @ ref.M @ v - exact) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7])
def test_lift_gives_face_integrals_2d(N):
    # u^T M LIFT g = sum_f int_{-1}^{1} u g dxi (face parameter of length 2)
    ref = RefElement2D(N)
    xg, wg = special.roots_legendre(N + 2)
    faces = (lambda x: (x, -np.ones_like(x)), lambda x: (x, -x), lambda x: (-np.ones_like(x), x))
    rng = np.random.default_rng(N)
    for _ in range(4):
        a1, b1, a2, b2 = rng.integers(0, N + 1, 4)
        if a1 + b1 > N or a2 + b2 > N:
            continue
        u = ref.r ** a1 * ref.s ** b1
        v = ref.r ** a2 * ref.s ** b2
        g = np.concatenate([v[ref.Fmask[f]] for f in range(3)])
        lhs = u @ ref.M @ ref.LIFT @ g
        rhs = 0.0
        for f in range(3):
            rr, ss = faces[f](xg)
            rhs += np.dot(wg, rr ** (a1 + a2) * ss ** (b1 + b2))
        assert abs(lhs - rhs) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 4])
def test_lift_gives_face_integrals_3d(N):
    ref = RefElement3D(N)
    qu, qv, qw = _tri_quadrature(2 * N)
    one = np.ones_like(qu)
    # each face parametrised by the two coordinates the oracle uses for its face mass matrix
    faces = (lambda u, v: (u, v, -one), lambda u, v: (u, -one, v),
             lambda u, v: (-1 - u - v, u, v), lambda u, v: (-one, u, v))
    rng = np.random.default_rng(N)
    mons = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]
    for _ in range(4):
        m1, m2 = (mons[i] for i in rng.integers(0, len(mons), 2))
        u = ref.r ** m1[0] * ref.s ** m1[1] * ref.t ** m1[2]
        v = ref.r ** m2[0] * ref.s ** m2[1] * ref.t ** m2[2]
        g = np.concatenate([v[ref.Fmask[f]] for f in range(4)])
        lhs = u @ ref.M @ ref.LIFT @ g
        rhs = 0.0
        for f in range(4):
            rr, ss, tt = faces[f](qu, qv)
            rhs += np.dot(qw, rr ** (m1[0] + m2[0]) * ss ** (m1[1] + m2[1]) * tt ** (m1[2] + m2[2]))
        assert abs(lhs - rhs) < 1e-12


# ---------------------------------------------------------------- divergence theorem per element

@pytest.mark.parametrize("N", [1, 3, 5])
def test_divergence_theorem_2d(N):
    m = inputs.tri_grid(4, jitter=0.15, seed=11)
    d = Discretization2D(m.vx, m.vy, m.elem_verts, N)
    ref = d.ref
    rng = np.random.default_rng(N)
    u = rng.standard_normal((d.K, d.Np))
    uf = u.reshape(-1)[d.vmapM]
    for comp, (gr, gs, n) in enumerate(((d.rx, d.sx, d.nx), (d.ry, d.sy, d.ny))):
        du = gr[:, None] * (u @ ref.Dr.T) + gs[:, None] * (u @ ref.Ds.T)
        lhs = d.J * np.einsum("ki,ij,kj->k", np.ones_like(u), ref.M, du)
        surf = (d.Fscale * n * uf) @ ref.LIFT.T
        rhs = d.J * np.einsum("ki,ij,kj->k", np.ones_like(u), ref.M, surf)
        assert np.allclose(lhs, rhs, atol=1e-11 * np.abs(lhs).max())
    # geometric sanity: total area 4, outward normals on the square's boundary
    assert abs(np.sum(2 * d.J) - 4.0) < 1e-12
    b = d.boundary
    xb, yb = d.x.reshape(-1)[d.vmapM[b]], d.y.reshape(-1)[d.vmapM[b]]
    assert np.allclose(np.abs(d.nx[b]) + np.abs(d.ny[b]), 1.0)
    assert np.all(d.nx[b] * xb + d.ny[b] * yb > 0)


@pytest.mark.parametrize("N", [1, 2, 4])
def test_divergence_theorem_3d(N):
    m = inputs.tet_grid(2, jitter=0.1, seed=12)
    d = Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, N)
    ref = d.ref
    rng = np.random.default_rng(N)
    u = rng.standard_normal((d.K, d.Np))
    uf = u.reshape(-1)[d.vmapM]
    grads = ((d.rx, d.sx, d.tx, d.nx), (d.ry, d.sy, d.ty, d.ny), (d.rz, d.sz, d.tz, d.nz))
    for gr, gs, gt, n in grads:
        du = gr[:, None] * (u @ ref.Dr.T) + gs[:, None] * (u @ ref.Ds.T) + gt[:, None] * (u @ ref.Dt.T)
        lhs = d.J * (np.ones(d.Np) @ ref.M @ du.T)
        surf = (d.Fscale * n * uf) @ ref.LIFT.T
        rhs = d.J * (np.ones(d.Np) @ ref.M @ surf.T)
        assert np.allclose(lhs, rhs, atol=1e-11 * np.abs(lhs).max())
    assert abs(np.sum(d.J * 4 / 3) - 8.0) < 1e-12


def test_connectivity_structured_grid():
    s = 6
    m = inputs.tri_grid(s, seed=3, permute=True)
    d = Discretization2D(m.vx, m.vy, m.elem_verts, 2)
    nb = d.boundary[:, ::d.Nfp].sum()
    assert nb == 4 * s
    k = np.arange(d.K)[:, None]
    inner = ~d.boundary[:, ::d.Nfp]
    back = d.EToE[d.EToE, d.EToF]
    assert np.all(back[inner] == np.broadcast_to(k, back.shape)[inner])
    # matched face nodes coincide
    x, y = d.x.reshape(-1), d.y.reshape(-1)
    assert np.allclose(x[d.vmapM], x[d.vmapP]) and np.allclose(y[d.vmapM], y[d.vmapP])


def test_connectivity_tets():
    n = 3
    m = inputs.tet_grid(n, seed=4, permute=True)
    d = Discretization3D(m.vx, m.vy, m.vz, m.elem_verts, 2)
    # boundary faces: 6 sides * n^2 squares * 2 triangles
    assert d.boundary[:, ::d.Nfp].sum() == 12 * n * n
    X = [c.reshape(-1) for c in d.coords()]
    for c in X:
        assert np.allclose(c[d.vmapM], c[d.vmapP])
