"""Geometry and connectivity for the FP64 oracle (test infrastructure only).

Affine element maps and the local-to-global chain rule follow the paper's
"Implementation Aspects" (affine map Psi = A_k (r,s)^T + b_k, mass matrix
|A_k| M, eq. dg-diff-local-to-global).  Face quantities follow the surface
kernel's description in the "Minimal Implementation" section: outward unit
normal, and Fscale = surface Jacobian / volume Jacobian.

Face neighbours are found by matching the physical coordinates of face nodes
(vmapM / vmapP of the paper's CPU right-hand side), deliberately a different
route from the library's combinatorial one so that the two cross-check.
Boundary face nodes map to themselves and are flagged (the PEC wall).
"""

from __future__ import annotations

import numpy as np

from .element import RefElement2D, RefElement3D


def _match_faces(face_keys: np.ndarray):
    """Pair faces (rows of sorted global vertex ids) that share the same
    vertex set.  Returns the partner face index (or -1 on the boundary)."""
    F = face_keys.shape[0]
    order = np.lexsort(face_keys.T[::-1])
    sk = face_keys[order]
    same = np.all(sk[1:] == sk[:-1], axis=1)
    partner = -np.ones(F, dtype=np.int64)
    idx = np.nonzero(same)[0]
    partner[order[idx]] = order[idx + 1]
    partner[order[idx + 1]] = order[idx]
    # a vertex set shared by more than two faces is a non-conforming mesh
    if idx.size and np.any(np.diff(idx) == 1):
        raise ValueError("non-conforming mesh: a face is shared by >2 elements")
    return partner


def _coordinate_match(xM: np.ndarray, xP: np.ndarray, tol: float) -> np.ndarray:
    """For each pair of matched faces, the permutation taking the partner's
    face nodes onto ours, found by nearest coordinates.
    xM, xP: (F, Nfp, d).  Returns (F, Nfp) indices into the partner face."""
    F = xM.shape[0]
    out = np.empty(xM.shape[:2], dtype=np.int64)
    chunk = 65536
    for c0 in range(0, F, chunk):
        a = xM[c0:c0 + chunk]
        b = xP[c0:c0 + chunk]
        d2 = np.sum((a[:, :, None, :] - b[:, None, :, :]) ** 2, axis=-1)
        j = np.argmin(d2, axis=2)
        dmin = np.take_along_axis(d2, j[:, :, None], axis=2)[..., 0]
        if np.any(dmin > tol * tol):
            raise ValueError("face nodes do not match: non-conforming mesh")
        out[c0:c0 + chunk] = j
    return out


class Discretization2D:
    """Per-element geometry and face maps of a straight-sided triangle mesh.

    VX, VY: vertex coordinates; EToV: K x 3 vertex ids, counter-clockwise
    (positive Jacobian).  eps, mu: per-element material (default 1)."""

    def __init__(self, VX, VY, EToV, N: int, eps=None, mu=None):
        self.ref = ref = RefElement2D(N)
        VX = np.asarray(VX, dtype=np.float64)
        VY = np.asarray(VY, dtype=np.float64)
        EToV = np.asarray(EToV, dtype=np.int64)
        self.K = K = EToV.shape[0]
        self.Np, self.Nfp, self.Nfaces = ref.Np, ref.Nfp, 3
        K = self.K
        self.eps = np.ones(K) if eps is None else np.asarray(eps, dtype=np.float64).copy()
        self.mu = np.ones(K) if mu is None else np.asarray(mu, dtype=np.float64).copy()
        v = [EToV[:, i] for i in range(3)]
        x1, x2, x3 = (VX[vi][:, None] for vi in v)
        y1, y2, y3 = (VY[vi][:, None] for vi in v)
        r, s = ref.r[None, :], ref.s[None, :]
        # affine map from (-1,-1),(1,-1),(-1,1)
        self.x = 0.5 * (-(r + s) * x1 + (1 + r) * x2 + (1 + s) * x3)
        self.y = 0.5 * (-(r + s) * y1 + (1 + r) * y2 + (1 + s) * y3)
        xr = 0.5 * (VX[v[1]] - VX[v[0]])
        xs = 0.5 * (VX[v[2]] - VX[v[0]])
        yr = 0.5 * (VY[v[1]] - VY[v[0]])
        ys = 0.5 * (VY[v[2]] - VY[v[0]])
        J = xr * ys - xs * yr
        if np.any(J <= 0):
            raise ValueError("element with non-positive Jacobian")
        self.J = J
        # inverse of the affine Jacobian: entries of A_k^{-1}
        self.rx, self.ry = ys / J, -xs / J
        self.sx, self.sy = -yr / J, xr / J
        # faces: 1 = v1->v2, 2 = v2->v3, 3 = v3->v1 (counter-clockwise)
        face_verts = ((0, 1), (1, 2), (2, 0))
        nx = np.empty((K, 3))
        ny = np.empty((K, 3))
        sJ = np.empty((K, 3))
        for f, (a, b) in enumerate(face_verts):
            dx = VX[v[b]] - VX[v[a]]
            dy = VY[v[b]] - VY[v[a]]
            L = np.hypot(dx, dy)
            nx[:, f], ny[:, f] = dy / L, -dx / L   # outward for CCW elements
            sJ[:, f] = 0.5 * L
        Nfp = self.Nfp
        self.nx = np.repeat(nx, Nfp, axis=1)        # K x Nafp
        self.ny = np.repeat(ny, Nfp, axis=1)
        self.sJ = np.repeat(sJ, Nfp, axis=1)
        self.Fscale = self.sJ / J[:, None]
        self._connect(EToV, face_verts)

    def _connect(self, EToV, face_verts):
        K, Np, Nfp = self.K, self.Np, self.Nfp
        Nf = len(face_verts)
        keys = np.stack([np.sort(EToV[:, list(fv)], axis=1) for fv in face_verts], axis=1)
        keys = keys.reshape(K * Nf, -1)
        partner = _match_faces(keys)
        Fmask = self.ref.Fmask
        vmapM = (np.arange(K)[:, None, None] * Np + Fmask[None, :, :]).reshape(K * Nf, Nfp)
        coords = np.stack([c.reshape(-1) for c in self.coords()], axis=1)
        bnd = partner < 0
        pf = np.where(bnd, np.arange(K * Nf), partner)
        xM = coords[vmapM]
        xP = coords[vmapM[pf]]
        span = float(np.max(coords.max(axis=0) - coords.min(axis=0)))
        perm = _coordinate_match(xM, xP, 1e-9 * max(span, 1.0))
        vmapP = np.take_along_axis(vmapM[pf], perm, axis=1)
        self.vmapM = vmapM.reshape(K, Nf * Nfp)
        self.vmapP = vmapP.reshape(K, Nf * Nfp)
        self.boundary = np.repeat(bnd.reshape(K, Nf), Nfp, axis=1)  # K x Nafp
        self.EToE = np.where(bnd, np.repeat(np.arange(K), Nf), pf // Nf).reshape(K, Nf)
        self.EToF = np.where(bnd, np.tile(np.arange(Nf), K), pf % Nf).reshape(K, Nf)

    def coords(self):
        return (self.x, self.y)

    def inradius(self) -> np.ndarray:
        """r_in = 2 * area / perimeter per element."""
        area = 2.0 * self.J
        perim = 2.0 * self.sJ[:, ::self.Nfp].sum(axis=1)
        return 2.0 * area / perim


class Discretization3D:
    """Per-element geometry and face maps of a straight-sided tetrahedral
    mesh.  EToV: K x 4, positively oriented."""

    def __init__(self, VX, VY, VZ, EToV, N: int, eps=None, mu=None):
        self.ref = ref = RefElement3D(N)
        V = np.stack([np.asarray(VX, float), np.asarray(VY, float), np.asarray(VZ, float)], axis=1)
        EToV = np.asarray(EToV, dtype=np.int64)
        self.K = K = EToV.shape[0]
        self.Np, self.Nfp, self.Nfaces = ref.Np, ref.Nfp, 4
        self.eps = np.ones(K) if eps is None else np.asarray(eps, dtype=np.float64).copy()
        self.mu = np.ones(K) if mu is None else np.asarray(mu, dtype=np.float64).copy()
        P = [V[EToV[:, i]] for i in range(4)]            # each K x 3
        r, s, t = ref.r[None, :], ref.s[None, :], ref.t[None, :]
        lam = (-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2)
        self.x = sum(lam[i] * P[i][:, 0:1] for i in range(4))
        self.y = sum(lam[i] * P[i][:, 1:2] for i in range(4))
        self.z = sum(lam[i] * P[i][:, 2:3] for i in range(4))
        # affine Jacobian columns: d x / d(r,s,t)
        A = np.stack([(P[1] - P[0]) / 2, (P[2] - P[0]) / 2, (P[3] - P[0]) / 2], axis=2)  # K x 3 x 3
        J = np.linalg.det(A)
        if np.any(J <= 0):
            raise ValueError("element with non-positive Jacobian")
        self.J = J
        Ainv = np.linalg.inv(A)   # rows: grad r, grad s, grad t
        self.rx, self.ry, self.rz = Ainv[:, 0, 0], Ainv[:, 0, 1], Ainv[:, 0, 2]
        self.sx, self.sy, self.sz = Ainv[:, 1, 0], Ainv[:, 1, 1], Ainv[:, 1, 2]
        self.tx, self.ty, self.tz = Ainv[:, 2, 0], Ainv[:, 2, 1], Ainv[:, 2, 2]
        # faces in the reference order: t=-1, s=-1, r+s+t=-1, r=-1
        face_verts = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))
        opposite = (3, 2, 0, 1)
        n = np.empty((K, 4, 3))
        sJ = np.empty((K, 4))
        for f, (a, b, c) in enumerate(face_verts):
            cr = np.cross(P[b] - P[a], P[c] - P[a])
            into = np.einsum("ij,ij->i", cr, P[opposite[f]] - P[a])
            cr = np.where((into > 0)[:, None], -cr, cr)   # point away from the opposite vertex
            area2 = np.linalg.norm(cr, axis=1)
            n[:, f, :] = cr / area2[:, None]
            sJ[:, f] = area2 / 4.0   # physical area |cr|/2 over the reference face area 2
        Nfp = self.Nfp
        self.nx = np.repeat(n[:, :, 0], Nfp, axis=1)
        self.ny = np.repeat(n[:, :, 1], Nfp, axis=1)
        self.nz = np.repeat(n[:, :, 2], Nfp, axis=1)
        self.sJ = np.repeat(sJ, Nfp, axis=1)
        self.Fscale = self.sJ / J[:, None]
        Discretization2D._connect(self, EToV, face_verts)

    def coords(self):
        return (self.x, self.y, self.z)

    def inradius(self) -> np.ndarray:
        """r_in = 3 * volume / total face area per element."""
        vol = self.J * (4.0 / 3.0)
        area = 2.0 * self.sJ[:, ::self.Nfp].sum(axis=1)
        return 3.0 * vol / area
