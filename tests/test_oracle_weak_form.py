"""Brute-force pin of the oracle's strong-form operator against an
independently assembled weak form (CPU only).

The paper derives the semi-discrete scheme from the weak form of eq. dg-weak
(test with every basis function of an element, integrate the flux by parts,
replace the boundary flux by the numerical flux F*) and turns it into the
strong form of eqs. dg-strong and dg-strong-explicit by a second integration
by parts.  On straight-sided (affine) elements the two are the same operator
exactly, so the matrix of the oracle's `rhs` (assembled column by column from
unit vectors) must equal the matrix of the weak form built here from scratch:

  * a Lagrange basis on the element's nodes from a monomial Vandermonde (not
    the oracle's orthonormal basis, V, Dr, Ds, M or LIFT);
  * element mass and stiffness matrices M_ij = int l_i l_j and
    S_d,ij = int l_i d_d l_j by collapsed Gauss quadrature, through each
    element's affine map computed here from its vertices;
  * face integrals of n.F* l_i by Gauss quadrature on each physical face,
    the partner trace evaluated from the neighbour's polynomial at the same
    physical point (neighbours found here from shared vertices; no vmapM,
    vmapP, Fmask, normals or Fscale of the oracle);
  * the numerical flux of a linear hyperbolic system in Godunov form,
    n.F* = 1/2 A_n (q- + q+) + alpha/2 |A_n| (q- - q+), with A_n the normal
    flux matrix of the PDE itself and |A_n| from its eigen-decomposition
    (the exact upwind flux at alpha = 1, the central flux at alpha = 0);
  * the PEC wall as the mirror state H+ = H-, E+ = -E-.

Planted mistakes in the oracle (a dropped factor 1/2 in the flux, a flipped
sign of the surface term, Fscale without the 1/J) must break the agreement.
"""

import math

import numpy as np
import pytest
from scipy import special

import oracle.maxwell as om
from oracle import Discretization2D, Discretization3D, Maxwell2D, Maxwell3D
from paper_1304_5546_amd import inputs


# ---------------------------------------------------------------- quadrature on the reference simplices

def _tri_rule(deg):
    n = deg // 2 + 2
    xa, wa = special.roots_legendre(n)
    xb, wb = special.roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(xa, xb, indexing="ij")
    W = np.outer(wa, wb) * 0.5
    return ((1 + A) * (1 - B) / 2 - 1).ravel(), B.ravel(), W.ravel()


def _tet_rule(deg):
    n = deg // 2 + 2
    xa, wa = special.roots_legendre(n)
    xb, wb = special.roots_jacobi(n, 1.0, 0.0)
    xc, wc = special.roots_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(xa, xb, xc, indexing="ij")
    W = wa[:, None, None] * wb[None, :, None] * wc[None, None, :] * 0.125
    r = (1 + A) * (1 - B) * (1 - C) / 4 - 1
    s = (1 + B) * (1 - C) / 2 - 1
    return r.ravel(), s.ravel(), C.ravel(), W.ravel()


# ---------------------------------------------------------------- Lagrange basis from monomials

class _Lagrange:
    """Lagrange basis of total degree N on the given nodes (rows of X, in
    reference coordinates), through the monomial Vandermonde."""

    def __init__(self, X, N):
        self.dim = X.shape[1]
        if self.dim == 2:
            self.exps = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
        else:
            self.exps = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a)
                         for c in range(N + 1 - a - b)]
        self.C = np.linalg.inv(self._mono(X))

    def _mono(self, X, d=None):
        cols = []
        for e in self.exps:
            v = np.ones(X.shape[0])
            coef = 1.0
            for k in range(self.dim):
                p = e[k] - (1 if d == k else 0)
                if d == k:
                    coef *= e[k]
                v = v * (X[:, k] ** p if p >= 0 else 0.0)
            cols.append(coef * v)
        return np.stack(cols, 1)

    def value(self, X):
        return self._mono(X) @ self.C

    def grad(self, X):
        return [self._mono(X, d) @ self.C for d in range(self.dim)]


# ---------------------------------------------------------------- PDE flux matrices (q_t + sum_d d_d (A_d q) = 0)

def _flux_matrices(dim):
    if dim == 2:
        # q = (Hx, Hy, Ez):  Hx_t = -Ez_y,  Hy_t = Ez_x,  Ez_t = Hy_x - Hx_y
        Ax = np.array([[0, 0, 0], [0, 0, -1], [0, -1, 0]], float)
        Ay = np.array([[0, 0, 1], [0, 0, 0], [1, 0, 0]], float)
        return [Ax, Ay]
    # q = (H, E):  H_t = -curl E,  E_t = curl H;  curl u = sum_d d_d (e_d x u)
    out = []
    for d in range(3):
        e = np.zeros(3)
        e[d] = 1.0
        X = np.array([[0, -e[2], e[1]], [e[2], 0, -e[0]], [-e[1], e[0], 0]])  # u -> e x u
        A = np.zeros((6, 6))
        A[0:3, 3:6] = X
        A[3:6, 0:3] = -X
        out.append(A)
    return out


def _godunov(An, alpha):
    lam, R = np.linalg.eigh(An)
    absA = (R * np.abs(lam)) @ R.T
    return 0.5 * An, 0.5 * alpha * absA


def _mirror(dim):
    return np.diag([1, 1, -1.0]) if dim == 2 else np.diag([1, 1, 1, -1, -1, -1.0])


# ---------------------------------------------------------------- weak-form assembly

class WeakForm:
    """The weak-form operator q -> dq/dt of the DG scheme on a small mesh."""

    def __init__(self, verts, EToV, nodes, N, alpha):
        self.V = np.asarray(verts, float)          # n_verts x dim
        self.EToV = np.asarray(EToV, int)
        self.dim = dim = self.V.shape[1]
        self.K = self.EToV.shape[0]
        self.basis = _Lagrange(nodes, N)
        self.Np = nodes.shape[0]
        self.nf = 3 if dim == 2 else 6
        self.Ad = _flux_matrices(dim)
        self.alpha = alpha
        self.mirror = _mirror(dim)
        if dim == 2:
            qr, qs, qw = _tri_rule(2 * N + 2)
            self.vq, self.vw = np.stack([qr, qs], 1), qw
            self.faces = ((0, 1), (1, 2), (2, 0))
            xg, wg = special.roots_legendre(N + 2)
            self.fq, self.fw = xg, wg
        else:
            qr, qs, qt, qw = _tet_rule(2 * N + 2)
            self.vq, self.vw = np.stack([qr, qs, qt], 1), qw
            self.faces = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))
            fr, fs, fw = _tri_rule(2 * N + 2)
            self.fq, self.fw = np.stack([fr, fs], 1), fw
        self._maps()
        self._neighbours()

    def _maps(self):
        self.A, self.Ainv, self.J, self.v0 = [], [], [], []
        for k in range(self.K):
            P = self.V[self.EToV[k]]
            A = np.stack([(P[i + 1] - P[0]) / 2 for i in range(self.dim)], 1)
            self.A.append(A)
            self.Ainv.append(np.linalg.inv(A))
            self.J.append(np.linalg.det(A))
            self.v0.append(P[0])
        assert min(self.J) > 0

    def _to_ref(self, k, X):
        return (X - self.v0[k]) @ self.Ainv[k].T - 1.0

    def _neighbours(self):
        owner = {}
        for k in range(self.K):
            for f, fv in enumerate(self.faces):
                key = tuple(sorted(self.EToV[k][list(fv)]))
                owner.setdefault(key, []).append(k)
        self.nbr = [[None] * len(self.faces) for _ in range(self.K)]
        for k in range(self.K):
            for f, fv in enumerate(self.faces):
                others = [e for e in owner[tuple(sorted(self.EToV[k][list(fv)]))] if e != k]
                assert len(others) <= 1
                self.nbr[k][f] = others[0] if others else None

    def _face(self, k, f):
        """Quadrature points (physical), weights (physical measure) and the
        outward unit normal of face f of element k."""
        P = self.V[self.EToV[k]]
        fv = self.faces[f]
        opp = [i for i in range(self.dim + 1) if i not in fv][0]
        if self.dim == 2:
            a, b = P[fv[0]], P[fv[1]]
            X = 0.5 * (1 - self.fq)[:, None] * a + 0.5 * (1 + self.fq)[:, None] * b
            length = np.linalg.norm(b - a)
            w = self.fw * length / 2
            t = (b - a) / length
            n = np.array([t[1], -t[0]])
        else:
            a, b, c = P[fv[0]], P[fv[1]], P[fv[2]]
            u, v = self.fq[:, 0], self.fq[:, 1]
            X = a + np.outer((u + 1) / 2, b - a) + np.outer((v + 1) / 2, c - a)
            cr = np.cross(b - a, c - a)
            w = self.fw * np.linalg.norm(cr) / 4
            n = cr / np.linalg.norm(cr)
        if np.dot(n, P[opp] - P[fv[0]]) > 0:
            n = -n
        return X, w, n

    def apply(self, q):
        """q: nf x K x Np nodal values -> dq/dt, same shape."""
        out = np.empty_like(q)
        ell_v = self.basis.value(self.vq)                       # nq x Np
        dref = self.basis.grad(self.vq)                         # dim x (nq x Np)
        for k in range(self.K):
            J, Ainv = self.J[k], self.Ainv[k]
            M = J * (ell_v.T * self.vw) @ ell_v
            # physical gradient of l_j at the quadrature points: A^-T grad_ref
            dphys = [sum(Ainv[e, d] * dref[e] for e in range(self.dim)) for d in range(self.dim)]
            b = np.zeros((self.nf, self.Np))
            for d in range(self.dim):
                S = J * (ell_v.T * self.vw) @ dphys[d]          # S_ij = int l_i d_d l_j
                F = self.Ad[d] @ q[:, k, :]                     # nf x Np nodal flux
                b += F @ S                                      # (S^T F_c)_i for each field c
            for f in range(len(self.faces)):
                X, w, n = self._face(k, f)
                lm = self.basis.value(self._to_ref(k, X))        # ng x Np
                qm = q[:, k, :] @ lm.T                           # nf x ng
                kp = self.nbr[k][f]
                if kp is None:
                    qp = self.mirror @ qm
                else:
                    qp = q[:, kp, :] @ self.basis.value(self._to_ref(kp, X)).T
                An = sum(n[d] * self.Ad[d] for d in range(self.dim))
                C, D = _godunov(An, self.alpha)
                Fstar = C @ (qm + qp) + D @ (qm - qp)            # nf x ng
                b -= (Fstar * w) @ lm                            # int n.F* l_i
            out[:, k, :] = np.linalg.solve(M, b.T).T
        return out


def _matrix(apply, nf, K, Np):
    n = nf * K * Np
    L = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        L[:, j] = apply(e.reshape(nf, K, Np)).reshape(-1)
    return L


def _generic_affine(dim, seed):
    rng = np.random.default_rng(seed)
    A = np.eye(dim) + 0.3 * rng.standard_normal((dim, dim))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    return A, rng.standard_normal(dim)


def _mesh2d(seed=21):
    m = inputs.tri_grid(2, jitter=0.15, seed=seed)          # 8 triangles
    A, c = _generic_affine(2, seed)
    X = np.stack([m.vx, m.vy], 1) @ A.T + c
    return X, m.elem_verts


def _mesh3d(seed=22):
    m = inputs.tet_grid(1, seed=seed)                        # 6 tetrahedra
    A, c = _generic_affine(3, seed)
    X = np.stack([m.vx, m.vy, m.vz], 1) @ A.T + c
    return X, m.elem_verts


def _strong_vs_weak_2d(N, alpha, make_op=Maxwell2D):
    X, ev = _mesh2d()
    d = Discretization2D(X[:, 0], X[:, 1], ev, N)
    op = make_op(d, alpha)
    wf = WeakForm(X, ev, np.stack([d.ref.r, d.ref.s], 1), N, alpha)
    Ls = _matrix(op.rhs, 3, d.K, d.Np)
    Lw = _matrix(wf.apply, 3, d.K, d.Np)
    return float(np.abs(Ls - Lw).max() / np.abs(Lw).max())


def _strong_vs_weak_3d(N, alpha, make_op=Maxwell3D):
    X, ev = _mesh3d()
    d = Discretization3D(X[:, 0], X[:, 1], X[:, 2], ev, N)
    op = make_op(d, alpha)
    wf = WeakForm(X, ev, np.stack([d.ref.r, d.ref.s, d.ref.t], 1), N, alpha)
    Ls = _matrix(op.rhs, 6, d.K, d.Np)
    Lw = _matrix(wf.apply, 6, d.K, d.Np)
    return float(np.abs(Ls - Lw).max() / np.abs(Lw).max())


# ---------------------------------------------------------------- pins

def test_weak_form_helpers_are_sound():
    # Godunov flux of the 2D system at alpha = 1 is the exact upwind flux:
    # A+ q- + A- q+ with A+- the positive/negative parts of A_n
    rng = np.random.default_rng(1)
    n = rng.standard_normal(2)
    n /= np.linalg.norm(n)
    An = sum(n[d] * _flux_matrices(2)[d] for d in range(2))
    lam, R = np.linalg.eigh(An)
    assert np.allclose(sorted(lam), [-1, 0, 1])             # wave speeds +-1 and 0
    Ap = (R * np.maximum(lam, 0)) @ R.T
    Am = (R * np.minimum(lam, 0)) @ R.T
    C, D = _godunov(An, 1.0)
    qm, qp = rng.standard_normal(3), rng.standard_normal(3)
    assert np.allclose(C @ (qm + qp) + D @ (qm - qp), Ap @ qm + Am @ qp, atol=1e-14)
    # consistency: F*(q, q) = A_n q for any alpha
    C, D = _godunov(An, 0.37)
    assert np.allclose(C @ (2 * qm), An @ qm, atol=1e-14)
    # the 3D system: speeds +-1 (twice each) and 0 (twice)
    n3 = rng.standard_normal(3)
    n3 /= np.linalg.norm(n3)
    A3 = sum(n3[d] * _flux_matrices(3)[d] for d in range(3))
    assert np.allclose(sorted(np.linalg.eigvalsh(A3)), [-1, -1, 0, 0, 1, 1], atol=1e-14)
    # the weak-form element maps tile the mapped square: total area 4 det(A)
    X, ev = _mesh2d()
    A, _ = _generic_affine(2, 21)
    nodes = np.array([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])
    wf = WeakForm(X, ev, nodes, 1, 1.0)
    assert abs(2.0 * sum(wf.J) - 4.0 * np.linalg.det(A)) < 1e-13
    # its mass matrix integrates the linear function x + 2y exactly per element
    ell = wf.basis.value(wf.vq)
    for k in range(wf.K):
        P = wf.V[wf.EToV[k]]
        u = P[:, 0] + 2 * P[:, 1]                   # nodal values at the vertices (N = 1)
        M = wf.J[k] * (ell.T * wf.vw) @ ell
        exact = wf.J[k] * 2.0 * u.mean()            # area times the value at the centroid
        assert abs(np.ones(3) @ M @ u - exact) < 1e-13 * max(1.0, abs(exact))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
def test_strong_form_equals_weak_form_2d(N, alpha):
    err = _strong_vs_weak_2d(N, alpha)
    print(f"2D N={N} alpha={alpha}: max |L_strong - L_weak| / max |L| = {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3])
@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_strong_form_equals_weak_form_3d(N, alpha):
    err = _strong_vs_weak_3d(N, alpha)
    print(f"3D N={N} alpha={alpha}: max |L_strong - L_weak| / max |L| = {err:.2e}")
    assert err < 1e-12


# ---------------------------------------------------------------- planted mistakes must fail the pin

def test_dropped_half_in_flux_is_caught(monkeypatch):
    true_flux = om.upwind_flux_2d

    def doubled(*a):
        return tuple(2.0 * x for x in true_flux(*a))
    monkeypatch.setattr(om, "upwind_flux_2d", doubled)
    assert _strong_vs_weak_2d(2, 1.0) > 1e-3
    true3 = om.upwind_flux_3d
    monkeypatch.setattr(om, "upwind_flux_3d", lambda *a: tuple(2.0 * x for x in true3(*a)))
    assert _strong_vs_weak_3d(1, 1.0) > 1e-3


def test_flipped_surface_sign_is_caught(monkeypatch):
    true_flux = om.upwind_flux_2d
    monkeypatch.setattr(om, "upwind_flux_2d", lambda *a: tuple(-x for x in true_flux(*a)))
    assert _strong_vs_weak_2d(2, 1.0) > 1e-3


def test_fscale_without_volume_jacobian_is_caught():
    class NoJ(Maxwell2D):
        def __init__(self, d, alpha):
            super().__init__(d, alpha)
            d.Fscale = d.sJ.copy()
    assert _strong_vs_weak_2d(2, 1.0, make_op=NoJ) > 1e-3


def test_dropped_upwind_dissipation_is_caught(monkeypatch):
    # the oracle run with alpha = 0 while the weak form uses alpha = 1
    X, ev = _mesh2d()
    d = Discretization2D(X[:, 0], X[:, 1], ev, 2)
    wf = WeakForm(X, ev, np.stack([d.ref.r, d.ref.s], 1), 2, 1.0)
    Ls = _matrix(Maxwell2D(d, 0.0).rhs, 3, d.K, d.Np)
    Lw = _matrix(wf.apply, 3, d.K, d.Np)
    assert np.abs(Ls - Lw).max() / np.abs(Lw).max() > 1e-3
    assert math.isfinite(float(np.abs(Lw).max()))
