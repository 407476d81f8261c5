"""Reference elements for the FP64 oracle (test infrastructure only).

The paper expands fields in Lagrange polynomials of total degree N on
stability-optimised nodes (section "Construction of the Method", citing
Warburton 2006) and builds the mass and differentiation matrices from
orthogonal polynomials on the simplex (section "Implementation Aspects",
Koornwinder-Dubiner), the combined face mass matrix of eq. dg-lift and
LIFT = M^{-1} M^{dI}.

Conventions (shared with the library only as a documented interface, not as
code):
  * 2D reference triangle with vertices (-1,-1), (1,-1), (-1,1); faces
    1: s=-1, 2: r+s=0, 3: r=-1.
  * 3D reference tetrahedron with vertices (-1,-1,-1), (1,-1,-1), (-1,1,-1),
    (-1,-1,1); faces 1: t=-1, 2: s=-1, 3: r+s+t=-1, 4: r=-1.
  * Node order inside an element: lattice order of the equispaced set the
    warp & blend map starts from, 2D: for j (s index) in 0..N, for i (r index)
    in 0..N-j; 3D: for k (t) in 0..N, for j (s) in 0..N-k, for i (r) in
    0..N-j-k.
  * Node set: warp & blend with the blend parameter ``alpha_opt(N)`` below.

The modal basis here uses SciPy's Jacobi polynomials normalised by their
closed-form norm (a library primitive), not a hand-written recurrence.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import special

# Warp & blend blend-parameter (Warburton 2006), 2D N=1..8 and 3D N=1..8.
# A shared input of the method (both implementations must use the same value
# for nodal parity); exactness and convergence hold for any value.
ALPHA_OPT_2D = {1: 0.0, 2: 0.0, 3: 1.4152, 4: 0.1001, 5: 0.2751, 6: 0.9800,
                7: 1.0999, 8: 1.2832}
ALPHA_OPT_3D = {1: 0.0, 2: 0.0, 3: 0.0, 4: 0.1002, 5: 1.1332, 6: 1.5608,
                7: 1.3413, 8: 1.2577}


# --------------------------------------------------------------------------
# 1D: orthonormal Jacobi polynomials, Gauss-Lobatto-Legendre nodes
# --------------------------------------------------------------------------

def _jacobi_norm2(n: int, a: float, b: float) -> float:
    """Squared L2 norm of the classical Jacobi polynomial P_n^(a,b) under
    the weight (1-x)^a (1+x)^b on [-1,1] (closed form)."""
    return (2.0 ** (a + b + 1) / (2 * n + a + b + 1)
            * math.gamma(n + a + 1) * math.gamma(n + b + 1)
            / (math.gamma(n + a + b + 1) * math.factorial(n)))


def jacobi(n: int, a: float, b: float, x: np.ndarray) -> np.ndarray:
    """Orthonormal Jacobi polynomial of degree n at x."""
    x = np.asarray(x, dtype=np.float64)
    return special.eval_jacobi(n, a, b, x) / math.sqrt(_jacobi_norm2(n, a, b))


def jacobi_deriv(n: int, a: float, b: float, x: np.ndarray) -> np.ndarray:
    """d/dx of the orthonormal Jacobi polynomial, from
    d/dx P_n^(a,b) = (n+a+b+1)/2 P_{n-1}^(a+1,b+1)."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    dp = 0.5 * (n + a + b + 1) * special.eval_jacobi(n - 1, a + 1, b + 1, x)
    return dp / math.sqrt(_jacobi_norm2(n, a, b))


def lgl_nodes(N: int) -> np.ndarray:
    """Legendre-Gauss-Lobatto nodes of degree N on [-1,1], ascending: the
    endpoints plus the zeros of P_N', which are the Gauss-Jacobi(1,1) points."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner, _ = special.roots_jacobi(N - 1, 1.0, 1.0)
    return np.concatenate(([-1.0], np.sort(inner), [1.0]))


def _warp_factor(N: int, x: np.ndarray) -> np.ndarray:
    """Edge warp of Warburton's construction: the interpolant (on N+1
    equispaced points) of the displacement from equispaced to LGL points,
    divided by (1-x^2).  Set to 0 at x = +-1, where the displacement and
    every blend that multiplies it vanish."""
    x = np.asarray(x, dtype=np.float64)
    xeq = np.linspace(-1.0, 1.0, N + 1)
    disp = lgl_nodes(N) - xeq
    w = np.zeros_like(x)
    for i in range(N + 1):
        li = np.ones_like(x)
        for j in range(N + 1):
            if j != i:
                li = li * (x - xeq[j]) / (xeq[i] - xeq[j])
        w = w + disp[i] * li
    inside = np.abs(x) < 1.0 - 1e-10
    out = np.zeros_like(x)
    out[inside] = w[inside] / (1.0 - x[inside] ** 2)
    return out


def _triangle_shift(N: int, alpha: float, La, Lb, Lc):
    """2D warp & blend displacement in the equilateral frame whose 'top'
    vertex carries La, 'left' vertex Lb and 'right' vertex Lc (side 2).
    Each edge contributes 4 * (product of its two barycentrics) * warp
    (of the difference of those barycentrics) * (1 + (alpha * opposite)^2)
    along the edge's direction."""
    c2, s2 = math.cos(2 * math.pi / 3), math.sin(2 * math.pi / 3)
    c4, s4 = math.cos(4 * math.pi / 3), math.sin(4 * math.pi / 3)
    # (opposite, from, to, direction from 'from'-vertex to 'to'-vertex)
    edges = ((La, Lb, Lc, (1.0, 0.0)),     # left -> right
             (Lb, Lc, La, (c2, s2)),       # right -> top
             (Lc, La, Lb, (c4, s4)))       # top -> left
    dx = np.zeros_like(La)
    dy = np.zeros_like(La)
    for opp, lf, lt, (ex, ey) in edges:
        amount = 4.0 * lf * lt * _warp_factor(N, lt - lf) * (1.0 + (alpha * opp) ** 2)
        dx = dx + amount * ex
        dy = dy + amount * ey
    return dx, dy


def _barycentric_to_ref(Lam: np.ndarray, ref_vertices: np.ndarray) -> np.ndarray:
    return Lam @ ref_vertices


def _cartesian_to_barycentric(P: np.ndarray, verts: np.ndarray) -> np.ndarray:
    """Barycentric coordinates of points P (n x d) in the simplex verts
    ((d+1) x d) by solving the (d+1)x(d+1) affine system."""
    d = verts.shape[1]
    A = np.vstack([verts.T, np.ones(d + 1)])
    rhs = np.vstack([P.T, np.ones(P.shape[0])])
    return np.linalg.solve(A, rhs).T


REF_TRI = np.array([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])
REF_TET = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0],
                    [-1.0, -1.0, 1.0]])


def equispaced_lattice_2d(N: int) -> np.ndarray:
    """Integer lattice (i, j), i+j <= N, in the documented node order."""
    return np.array([(i, j) for j in range(N + 1) for i in range(N + 1 - j)], dtype=np.int64)


def equispaced_lattice_3d(N: int) -> np.ndarray:
    return np.array([(i, j, k) for k in range(N + 1) for j in range(N + 1 - k)
                     for i in range(N + 1 - j - k)], dtype=np.int64)


def nodes_2d(N: int, alpha: float | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Warp & blend nodes on the reference triangle (Warburton 2006)."""
    alpha = ALPHA_OPT_2D[N] if alpha is None else alpha
    lat = equispaced_lattice_2d(N)
    # barycentrics w.r.t. reference vertices v1=(-1,-1), v2=(1,-1), v3=(-1,1)
    l2 = lat[:, 0] / N
    l3 = lat[:, 1] / N
    l1 = 1.0 - l2 - l3
    # equilateral triangle: v3 on top, v1 left, v2 right
    eq = np.array([[-1.0, -1.0 / math.sqrt(3.0)], [1.0, -1.0 / math.sqrt(3.0)],
                   [0.0, 2.0 / math.sqrt(3.0)]])
    P = np.stack([l1, l2, l3], axis=1) @ eq
    dx, dy = _triangle_shift(N, alpha, l3, l1, l2)
    P = P + np.stack([dx, dy], axis=1)
    lam = _cartesian_to_barycentric(P, eq)
    rs = _barycentric_to_ref(lam, REF_TRI)
    return rs[:, 0].copy(), rs[:, 1].copy()


def nodes_3d(N: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Warp & blend nodes on the reference tetrahedron (Warburton 2006):
    each face receives the 2D warp of its own barycentrics, blended into the
    volume by  lb*lc*ld / ((lb+la/2)(lc+la/2)(ld+la/2)) * (1+(alpha*la)^2)
    where la vanishes on the face; nodes on an edge of the face take the
    face warp itself."""
    alpha = ALPHA_OPT_3D[N]
    lat = equispaced_lattice_3d(N)
    lam = np.empty((lat.shape[0], 4))
    lam[:, 1] = lat[:, 0] / N
    lam[:, 2] = lat[:, 1] / N
    lam[:, 3] = lat[:, 2] / N
    lam[:, 0] = 1.0 - lam[:, 1] - lam[:, 2] - lam[:, 3]
    s3, s6 = math.sqrt(3.0), math.sqrt(6.0)
    eq = np.array([[-1.0, -1.0 / s3, -1.0 / s6], [1.0, -1.0 / s3, -1.0 / s6],
                   [0.0, 2.0 / s3, -1.0 / s6], [0.0, 0.0, 3.0 / s6]])
    P = lam @ eq
    shift = np.zeros_like(P)
    tol = 1e-10
    # face = (vertex opposite the face, (top, left, right) vertices of the face)
    faces = ((3, (2, 0, 1)), (2, (3, 0, 1)), (0, (3, 1, 2)), (1, (3, 0, 2)))
    for opp, (vt, vl, vr) in faces:
        la, lt, ll, lr = lam[:, opp], lam[:, vt], lam[:, vl], lam[:, vr]
        wx, wy = _triangle_shift(N, alpha, lt, ll, lr)
        t1 = eq[vr] - eq[vl]
        t1 /= np.linalg.norm(t1)
        t2 = eq[vt] - 0.5 * (eq[vl] + eq[vr])
        t2 /= np.linalg.norm(t2)
        blend = lt * ll * lr
        denom = (lt + 0.5 * la) * (ll + 0.5 * la) * (lr + 0.5 * la)
        ok = denom > tol
        blend = np.where(ok, (1.0 + (alpha * la) ** 2) * blend / np.where(ok, denom, 1.0), blend)
        face_warp = np.outer(wx, t1) + np.outer(wy, t2)
        shift += blend[:, None] * face_warp
        on_face_edge = (la < tol) & (((lt > tol).astype(int) + (ll > tol) + (lr > tol)) < 3)
        shift[on_face_edge] = face_warp[on_face_edge]
    P = P + shift
    lam2 = _cartesian_to_barycentric(P, eq)
    rst = _barycentric_to_ref(lam2, REF_TET)
    return rst[:, 0].copy(), rst[:, 1].copy(), rst[:, 2].copy()


# --------------------------------------------------------------------------
# Orthonormal (Koornwinder-Dubiner) bases and their gradients
# --------------------------------------------------------------------------

def _pos_pow(x: np.ndarray, p: int) -> np.ndarray:
    """x**p for p >= 0; for p < 0 returns zeros (only reached where the
    multiplying coefficient is identically zero)."""
    if p < 0:
        return np.zeros_like(x)
    return x ** p


def _collapse_2d(r, s):
    denom = 1.0 - s
    a = np.where(np.abs(denom) > 1e-14, 2.0 * (1.0 + r) / np.where(np.abs(denom) > 1e-14, denom, 1.0) - 1.0, -1.0)
    return a, s


def basis_2d(N: int, r, s):
    """Orthonormal basis on the reference triangle and its (r, s) gradient:
    psi_ij = sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i, a = 2(1+r)/(1-s)-1, b = s."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    a, b = _collapse_2d(r, s)
    V, Vr, Vs = [], [], []
    for i in range(N + 1):
        for j in range(N + 1 - i):
            A, dA = jacobi(i, 0, 0, a), jacobi_deriv(i, 0, 0, a)
            B0, dB0 = jacobi(j, 2 * i + 1, 0, b), jacobi_deriv(j, 2 * i + 1, 0, b)
            psi = math.sqrt(2.0) * A * B0 * _pos_pow(1 - b, i)
            # d/dr = 2/(1-b) d/da ;  d/ds = (1+a)/(1-b) d/da + d/db
            dpsi_a_over = math.sqrt(2.0) * dA * B0 * _pos_pow(1 - b, i - 1)  # (d psi/da)/(1-b)
            dB = dB0 * _pos_pow(1 - b, i) - i * B0 * _pos_pow(1 - b, i - 1)
            dpsi_b = math.sqrt(2.0) * A * dB
            V.append(psi)
            Vr.append(2.0 * dpsi_a_over)
            Vs.append((1 + a) * dpsi_a_over + dpsi_b)
    return np.stack(V, 1), np.stack(Vr, 1), np.stack(Vs, 1)


def basis_3d(N: int, r, s, t):
    """Orthonormal basis on the reference tetrahedron and its gradient:
    psi_ijk = 2 sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i P_k^(2i+2j+2,0)(c) (1-c)^(i+j),
    a = 2(1+r)/(-s-t) - 1, b = 2(1+s)/(1-t) - 1, c = t."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    d1 = -s - t
    a = np.where(np.abs(d1) > 1e-14, 2.0 * (1 + r) / np.where(np.abs(d1) > 1e-14, d1, 1.0) - 1.0, -1.0)
    d2 = 1.0 - t
    b = np.where(np.abs(d2) > 1e-14, 2.0 * (1 + s) / np.where(np.abs(d2) > 1e-14, d2, 1.0) - 1.0, -1.0)
    c = t
    k0 = 2.0 * math.sqrt(2.0)
    V, Vr, Vs, Vt = [], [], [], []
    for i in range(N + 1):
        for j in range(N + 1 - i):
            for k in range(N + 1 - i - j):
                A, dA = jacobi(i, 0, 0, a), jacobi_deriv(i, 0, 0, a)
                Pj, dPj = jacobi(j, 2 * i + 1, 0, b), jacobi_deriv(j, 2 * i + 1, 0, b)
                Pk, dPk = jacobi(k, 2 * i + 2 * j + 2, 0, c), jacobi_deriv(k, 2 * i + 2 * j + 2, 0, c)
                B = Pj * _pos_pow(1 - b, i)
                C = Pk * _pos_pow(1 - c, i + j)
                dB = dPj * _pos_pow(1 - b, i) - i * Pj * _pos_pow(1 - b, i - 1)
                dC = dPk * _pos_pow(1 - c, i + j) - (i + j) * Pk * _pos_pow(1 - c, i + j - 1)
                # terms with the 1/((1-b)(1-c)) and 1/(1-c) factors folded into powers
                ta = dA * Pj * _pos_pow(1 - b, i - 1) * Pk * _pos_pow(1 - c, i + j - 1)
                tb = A * dB * Pk * _pos_pow(1 - c, i + j - 1)
                V.append(k0 * A * B * C)
                Vr.append(k0 * 4.0 * ta)
                Vs.append(k0 * (2.0 * (1 + a) * ta + 2.0 * tb))
                Vt.append(k0 * (2.0 * (1 + a) * ta + (1 + b) * tb + A * B * dC))
    return np.stack(V, 1), np.stack(Vr, 1), np.stack(Vs, 1), np.stack(Vt, 1)


def basis_1d(N: int, x):
    x = np.asarray(x, dtype=np.float64)
    return np.stack([jacobi(n, 0, 0, x) for n in range(N + 1)], 1)


# --------------------------------------------------------------------------
# Reference elements
# --------------------------------------------------------------------------

class RefElement2D:
    """Nodal reference triangle of order N: nodes, V, Dr, Ds, M, Fmask, LIFT."""

    Nfaces = 3

    def __init__(self, N: int):
        if not 1 <= N <= 8:
            raise ValueError("order N must be in 1..8")
        self.N = N
        self.Np = (N + 1) * (N + 2) // 2
        self.Nfp = N + 1
        self.r, self.s = nodes_2d(N)
        self.V, Vr, Vs = basis_2d(N, self.r, self.s)
        Vinv = np.linalg.inv(self.V)
        self.Dr = Vr @ Vinv                      # differentiation along r
        self.Ds = Vs @ Vinv
        self.M = np.linalg.inv(self.V @ self.V.T)  # reference mass matrix
        tol = 1e-10
        self.Fmask = np.array([
            np.nonzero(np.abs(self.s + 1) < tol)[0],
            np.nonzero(np.abs(self.r + self.s) < tol)[0],
            np.nonzero(np.abs(self.r + 1) < tol)[0],
        ])
        # combined face mass matrix M^{dI} (eq. dg-lift): 1D mass on the face
        # parameter in [-1,1] for every face
        face_param = (self.r, self.r, self.s)
        E = np.zeros((self.Np, self.Nfaces * self.Nfp))
        for f in range(self.Nfaces):
            x1 = face_param[f][self.Fmask[f]]
            V1 = basis_1d(N, x1)
            Mf = np.linalg.inv(V1 @ V1.T)
            E[np.ix_(self.Fmask[f], np.arange(f * self.Nfp, (f + 1) * self.Nfp))] = Mf
        self.Emat = E
        self.LIFT = self.V @ (self.V.T @ E)      # M^{-1} M^{dI}


class RefElement3D:
    """Nodal reference tetrahedron of order N: nodes, V, Dr, Ds, Dt, M, Fmask, LIFT."""

    Nfaces = 4

    def __init__(self, N: int):
        if not 1 <= N <= 8:
            raise ValueError("order N must be in 1..8")
        self.N = N
        self.Np = (N + 1) * (N + 2) * (N + 3) // 6
        self.Nfp = (N + 1) * (N + 2) // 2
        self.r, self.s, self.t = nodes_3d(N)
        self.V, Vr, Vs, Vt = basis_3d(N, self.r, self.s, self.t)
        Vinv = np.linalg.inv(self.V)
        self.Dr = Vr @ Vinv
        self.Ds = Vs @ Vinv
        self.Dt = Vt @ Vinv
        self.M = np.linalg.inv(self.V @ self.V.T)
        tol = 1e-10
        r, s, t = self.r, self.s, self.t
        self.Fmask = np.array([
            np.nonzero(np.abs(t + 1) < tol)[0],
            np.nonzero(np.abs(s + 1) < tol)[0],
            np.nonzero(np.abs(r + s + t + 1) < tol)[0],
            np.nonzero(np.abs(r + 1) < tol)[0],
        ])
        face_coords = ((r, s), (r, t), (s, t), (s, t))
        E = np.zeros((self.Np, self.Nfaces * self.Nfp))
        for f in range(self.Nfaces):
            u, v = face_coords[f]
            V2, _, _ = basis_2d(N, u[self.Fmask[f]], v[self.Fmask[f]])
            Mf = np.linalg.inv(V2 @ V2.T)
            E[np.ix_(self.Fmask[f], np.arange(f * self.Nfp, (f + 1) * self.Nfp))] = Mf
        self.Emat = E
        self.LIFT = self.V @ (self.V.T @ E)
