"""Seeded synthetic inputs: meshes of the PEC cavity and serving request mixes.

This module holds no arithmetic of the DG method.  It builds the inputs that
both the HIP library and the FP64 oracle consume (vertex coordinates, element
vertex lists, per-element materials, request parameters), each from a seeded
``numpy.random.Generator(PCG64(seed))``, with the draw order documented so the
inputs are reproducible.

The paper's only workload is a PEC cavity (section "A Precise Mathematical
Problem Statement"); its screenshot mesh is not published, so the cavity is
meshed here from a structured grid with jittered interior vertices.
"""

from __future__ import annotations

import hashlib
import itertools
from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    dim: int
    vx: np.ndarray            # float64 [n_verts]
    vy: np.ndarray
    vz: np.ndarray | None
    elem_verts: np.ndarray    # int32 [K, dim+1], positively oriented
    eps: np.ndarray | None = None   # float64 [K] or None (= 1)
    mu: np.ndarray | None = None

    @property
    def K(self) -> int:
        return int(self.elem_verts.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def tri_grid(s: int, jitter: float = 0.1, seed: int = 0, permute: bool = False) -> Mesh:
    """Square [-1,1]^2 meshed by an s x s grid, each cell split along its
    (i,j)-(i+1,j+1) diagonal into two counter-clockwise triangles (K = 2 s^2).

    Draw order: interior-vertex x offsets, then y offsets, each U(-jitter*h,
    jitter*h) with h = 2/s (boundary vertices stay on the square), then (if
    ``permute``) one ``permutation(K)`` of the element order."""
    rng = _rng(seed)
    h = 2.0 / s
    ii, jj = np.meshgrid(np.arange(s + 1), np.arange(s + 1), indexing="xy")
    vx = (-1.0 + h * ii).astype(np.float64).reshape(-1)
    vy = (-1.0 + h * jj).astype(np.float64).reshape(-1)
    interior = ((ii > 0) & (ii < s) & (jj > 0) & (jj < s)).reshape(-1)
    n_int = int(interior.sum())
    dx = rng.uniform(-jitter * h, jitter * h, n_int)
    dy = rng.uniform(-jitter * h, jitter * h, n_int)
    vx[interior] += dx
    vy[interior] += dy

    def vid(i, j):
        return j * (s + 1) + i

    ci, cj = np.meshgrid(np.arange(s), np.arange(s), indexing="xy")
    ci, cj = ci.reshape(-1), cj.reshape(-1)
    v00, v10 = vid(ci, cj), vid(ci + 1, cj)
    v11, v01 = vid(ci + 1, cj + 1), vid(ci, cj + 1)
    lower = np.stack([v00, v10, v11], axis=1)
    upper = np.stack([v00, v11, v01], axis=1)
    ev = np.stack([lower, upper], axis=1).reshape(-1, 3).astype(np.int32)
    if permute:
        ev = ev[rng.permutation(ev.shape[0])]
    return Mesh(2, vx, vy, None, np.ascontiguousarray(ev))


def tet_grid(n: int, jitter: float = 0.05, seed: int = 0, permute: bool = False) -> Mesh:
    """Cube [-1,1]^3 meshed by n^3 cubes, each split into 6 tetrahedra along
    its (0,0,0)-(1,1,1) diagonal (one per ordering of the three axes; the
    split is conforming), K = 6 n^3.  Vertex order is fixed so every
    tetrahedron is positively oriented.

    Draw order: interior-vertex x, y, z offsets, each U(-jitter*h, jitter*h),
    then (if ``permute``) ``permutation(K)``."""
    rng = _rng(seed)
    h = 2.0 / n
    # vertex id = (k*(n+1) + j)*(n+1) + i
    vid_all = np.arange((n + 1) ** 3)
    ii = vid_all % (n + 1)
    jj = (vid_all // (n + 1)) % (n + 1)
    kk = vid_all // (n + 1) ** 2
    vx = -1.0 + h * ii.astype(np.float64)
    vy = -1.0 + h * jj.astype(np.float64)
    vz = -1.0 + h * kk.astype(np.float64)
    interior = (ii > 0) & (ii < n) & (jj > 0) & (jj < n) & (kk > 0) & (kk < n)
    n_int = int(interior.sum())
    for arr in (vx, vy, vz):
        arr[interior] += rng.uniform(-jitter * h, jitter * h, n_int)

    def vid(i, j, k):
        return (k * (n + 1) + j) * (n + 1) + i

    cid = np.arange(n ** 3)          # cube id = (k*n + j)*n + i
    ci, cj, ck = cid % n, (cid // n) % n, cid // (n * n)
    tets = []
    for perm in itertools.permutations(range(3)):
        cur = np.zeros((3,), dtype=np.int64)
        path = [cur.copy()]
        for ax in perm:
            cur[ax] += 1
            path.append(cur.copy())
        ids = [vid(ci + p[0], cj + p[1], ck + p[2]) for p in path]
        # parity of the axis permutation decides the orientation of the path tet
        sign = np.linalg.det(np.array([path[1] - path[0], path[2] - path[0], path[3] - path[0]], float))
        if sign < 0:
            ids[2], ids[3] = ids[3], ids[2]
        tets.append(np.stack(ids, axis=1))
    ev = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    if permute:
        ev = ev[rng.permutation(ev.shape[0])]
    return Mesh(3, vx, vy, vz, np.ascontiguousarray(ev))


def disk_inclusion_eps(mesh: Mesh, center, radius: float, eps_in: float = 2.25) -> np.ndarray:
    """Per-element permittivity: eps_in where the element's vertex centroid
    lies in the disk, else 1 (a material input, not part of the method)."""
    ev = mesh.elem_verts
    cx = mesh.vx[ev].mean(axis=1)
    cy = mesh.vy[ev].mean(axis=1)
    inside = (cx - center[0]) ** 2 + (cy - center[1]) ** 2 < radius ** 2
    return np.where(inside, eps_in, 1.0)


@dataclass
class Request:
    index: int
    s: int
    order: int
    mode: tuple[int, int]
    disk_center: tuple[float, float]
    disk_radius: float
    t_final: float
    mesh_seed: int
    arrival: float = 0.0


def request_seed(master: int, i: int) -> int:
    """Per-request mesh seed: first 8 bytes of sha256(master, i)."""
    d = hashlib.sha256(f"{master}:{i}".encode()).digest()
    return int.from_bytes(d[:8], "little") & 0x7FFFFFFFFFFFFFFF


def make_requests(n: int = 256, seed: int = 4, s_range=(16, 256), orders=(3, 5, 7),
                  t_range=(0.5, 2.0)) -> list[Request]:
    """Serving mix.  Per request, in this draw order: s ~ U{s_range},
    N ~ U{orders}, (m, n) ~ U{1..4}^2, disk centre ~ U[-0.6,0.6]^2, disk
    radius ~ U[0.15,0.5], t_final ~ U[t_range]."""
    rng = _rng(seed)
    out = []
    for i in range(n):
        s = int(rng.integers(s_range[0], s_range[1] + 1))
        N = int(orders[int(rng.integers(0, len(orders)))])
        m_, n_ = (int(v) for v in rng.integers(1, 5, size=2))
        c = tuple(float(v) for v in rng.uniform(-0.6, 0.6, size=2))
        rad = float(rng.uniform(0.15, 0.5))
        tf = float(rng.uniform(t_range[0], t_range[1]))
        out.append(Request(i, s, N, (m_, n_), c, rad, tf, request_seed(seed, i)))
    return out


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate (per second)."""
    rng = _rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def request_mesh(req: Request, jitter: float = 0.1) -> Mesh:
    m = tri_grid(req.s, jitter=jitter, seed=req.mesh_seed)
    m.eps = disk_inclusion_eps(m, req.disk_center, req.disk_radius)
    m.mu = np.ones(m.K)
    return m
