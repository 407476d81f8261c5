"""Maxwell right-hand sides, LSRK4 time stepping and diagnostics for the FP64
oracle (test infrastructure only).

2D TM (eq. tm-maxwells, read with +dEz/dx in the Hy equation as the paper's
own CPU and GPU codes do):
    mu dHx/dt = -dEz/dy,   mu dHy/dt = dEz/dx,   eps dEz/dt = dHy/dx - dHx/dy.
3D: mu dH/dt = -curl E,  eps dE/dt = curl H.

Semi-discrete strong form (eq. dg-strong-explicit with the second derivative
read as d/dy): rhs = volume term + LIFT (Fscale * flux), the flux being the
paper's upwind flux n.(F - F*) (eq. max2d-numflux) with the factor 1/2 that
both of the paper's implementations apply, and jumps [q] = q^- - q^+.  The PEC
wall mirrors the state (E^+ = -E^-, H^+ = H^-), the paper's reflective
boundary condition.

Materials (piecewise-constant eps, mu; the paper sets them to 1) use the exact
upwind (Riemann) flux of the 1D problem normal to the face, impedance
Z = sqrt(mu/eps), tangential field h = nx Hy - ny Hx:
    flux_Ez = -([Ez] + Z+ [h]) / (Z- + Z+)
    flux_H  = (Z- [Ez] + Z- Z+ [h]) / (Z- + Z+) * (ny, -nx)
blended with the central flux (-[h]/2, [Ez]/2) by alpha, which reproduces the
paper's alpha-parametrised flux exactly when Z- = Z+ = 1; then
rhs_Ez += LIFT(Fscale flux_Ez)/eps-, rhs_H += LIFT(Fscale flux_H)/mu-.

Time stepping: the paper names only a "simple, explicit Runge-Kutta" method;
read as the five-stage fourth-order 2N-storage scheme of Carpenter and
Kennedy (1994): res = a_s res + dt L(q);  q = q + b_s res.
"""

from __future__ import annotations

import math

import numpy as np

from .element import lgl_nodes
from .mesh import Discretization2D, Discretization3D

# Carpenter & Kennedy (1994), five-stage fourth-order 2N-storage RK.
LSRK4_A = np.array([
    0.0,
    -567301805773.0 / 1357537059087.0,
    -2404267990393.0 / 2016746695238.0,
    -3550918686646.0 / 2091501179385.0,
    -1275806237668.0 / 842570457699.0,
])
LSRK4_B = np.array([
    1432997174477.0 / 9575080441755.0,
    5161836677717.0 / 13612068292357.0,
    1720146321549.0 / 2090206949498.0,
    3134564353537.0 / 4481467310338.0,
    2277821191437.0 / 14882151754819.0,
])
LSRK4_C = np.array([
    0.0,
    1432997174477.0 / 9575080441755.0,
    2526269341429.0 / 6820363962896.0,
    2006345519317.0 / 3224310063776.0,
    2802321613138.0 / 2924317926251.0,
])
LSRK4_FRACTIONS = (
    ((0, 1), (-567301805773, 1357537059087), (-2404267990393, 2016746695238),
     (-3550918686646, 2091501179385), (-1275806237668, 842570457699)),
    ((1432997174477, 9575080441755), (5161836677717, 13612068292357),
     (1720146321549, 2090206949498), (3134564353537, 4481467310338),
     (2277821191437, 14882151754819)),
)


def _eldot(Mat: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Apply the same small matrix to every element's nodal vector:
    u is K x n, result K x m = u @ Mat^T."""
    return u @ Mat.T


class _Base:
    def lsrk4_step(self, q: np.ndarray, res: np.ndarray, dt: float):
        """One full five-stage step, in place on (q, res)."""
        for s in range(5):
            rhs = self.rhs(q)
            res *= LSRK4_A[s]
            res += dt * rhs
            q += LSRK4_B[s] * res
        return q, res

    def run(self, q0: np.ndarray, dt: float, nsteps: int, energy_trace: bool = False):
        q = np.array(q0, dtype=np.float64, copy=True)
        res = np.zeros_like(q)
        energies = [self.energy(q)] if energy_trace else None
        for _ in range(nsteps):
            self.lsrk4_step(q, res, dt)
            if energy_trace:
                energies.append(self.energy(q))
        return (q, energies) if energy_trace else q

    def mass_inner(self, u: np.ndarray, v: np.ndarray) -> float:
        """sum_k J_k u_k^T M v_k for nodal fields u, v (K x Np)."""
        M = self.d.ref.M
        return float(np.sum(self.d.J * np.einsum("ki,ij,kj->k", u, M, v)))

    def rel_l2(self, q: np.ndarray, ref: np.ndarray) -> float:
        """Relative L2 (mass-matrix norm, unit field weights) of q - ref."""
        num = sum(self.mass_inner(q[f] - ref[f], q[f] - ref[f]) for f in range(q.shape[0]))
        den = sum(self.mass_inner(ref[f], ref[f]) for f in range(q.shape[0]))
        return math.sqrt(num / den)


def upwind_flux_2d(nx, ny, dHx, dHy, dEz, Zm, Zp, alpha):
    """Numerical flux n.(F - F*) of the 2D TM system at face nodes, from the
    jumps [q] = q^- - q^+: returns (flux_Hx, flux_Hy, flux_Ez) before the
    Fscale, 1/mu and 1/eps factors.  Exact upwind (Riemann) flux across a
    material interface with impedances Z-, Z+, blended by alpha with the
    central flux (F* = average)."""
    dh = nx * dHy - ny * dHx
    a = alpha
    fEz = (1 - a) * (-0.5 * dh) + a * (-(dEz + Zp * dh) / (Zm + Zp))
    fH = (1 - a) * (0.5 * dEz) + a * ((Zm * dEz + Zm * Zp * dh) / (Zm + Zp))
    return ny * fH, -nx * fH, fEz


def upwind_flux_3d(n, dH, dE, alpha):
    """Numerical flux of the 3D system (eps = mu = 1) from the jumps:
    flux_H = 1/2 ( n x [E] + alpha (n (n.[H]) - [H]) ),
    flux_E = 1/2 (-n x [H] + alpha (n (n.[E]) - [E]) ).
    n, dH, dE: arrays with the vector index first."""
    ndH = np.sum(n * dH, axis=0)
    ndE = np.sum(n * dE, axis=0)
    fH = 0.5 * (np.cross(n, dE, axis=0) + alpha * (n * ndH - dH))
    fE = 0.5 * (-np.cross(n, dH, axis=0) + alpha * (n * ndE - dE))
    return fH, fE


class Maxwell2D(_Base):
    """2D TM Maxwell on a Discretization2D.  Fields q = (Hx, Hy, Ez), each K x Np."""

    n_fields = 3

    def __init__(self, disc: Discretization2D, alpha: float = 1.0):
        self.d = disc
        self.alpha = float(alpha)
        d = disc
        Nfp = d.Nfp
        Zm = np.sqrt(d.mu / d.eps)
        ZM = Zm[:, None] * np.ones((1, 3 * Nfp))
        ZP = Zm.reshape(-1)[d.vmapP // d.Np]
        self.ZM, self.ZP = ZM, ZP   # boundary: Z+ = Z- (the mirror state)

    def rhs(self, q: np.ndarray) -> np.ndarray:
        d, ref = self.d, self.d.ref
        Hx, Hy, Ez = q
        # jumps [q] = q^- - q^+ at every face node
        dHx = Hx.flat[d.vmapM] - Hx.flat[d.vmapP]
        dHy = Hy.flat[d.vmapM] - Hy.flat[d.vmapP]
        dEz = Ez.flat[d.vmapM] - Ez.flat[d.vmapP]
        # PEC mirror state: H+ = H-, Ez+ = -Ez-
        b = d.boundary
        dHx[b] = 0.0
        dHy[b] = 0.0
        dEz[b] = 2.0 * Ez.flat[d.vmapM[b]]
        fluxHx, fluxHy, fEz = upwind_flux_2d(d.nx, d.ny, dHx, dHy, dEz,
                                             self.ZM, self.ZP, self.alpha)
        # local differentiation and the chain rule (eq. dg-diff-local-to-global)
        rx, ry, sx, sy = (g[:, None] for g in (d.rx, d.ry, d.sx, d.sy))
        Ezr, Ezs = _eldot(ref.Dr, Ez), _eldot(ref.Ds, Ez)
        Hxr, Hxs = _eldot(ref.Dr, Hx), _eldot(ref.Ds, Hx)
        Hyr, Hys = _eldot(ref.Dr, Hy), _eldot(ref.Ds, Hy)
        Ezx, Ezy = rx * Ezr + sx * Ezs, ry * Ezr + sy * Ezs
        Hyx = rx * Hyr + sx * Hys
        Hxy = ry * Hxr + sy * Hxs
        mu, eps = d.mu[:, None], d.eps[:, None]
        L, Fs = ref.LIFT, d.Fscale
        rhsHx = (-Ezy + _eldot(L, Fs * fluxHx)) / mu
        rhsHy = (Ezx + _eldot(L, Fs * fluxHy)) / mu
        rhsEz = (Hyx - Hxy + _eldot(L, Fs * fEz)) / eps
        return np.stack([rhsHx, rhsHy, rhsEz])

    def energy(self, q: np.ndarray) -> float:
        """0.5 * sum_k J_k (mu Hx^T M Hx + mu Hy^T M Hy + eps Ez^T M Ez)."""
        d, M = self.d, self.d.ref.M
        e = 0.0
        for f, w in ((0, d.mu), (1, d.mu), (2, d.eps)):
            e += float(np.sum(w * d.J * np.einsum("ki,ij,kj->k", q[f], M, q[f])))
        return 0.5 * e


class Maxwell3D(_Base):
    """3D Maxwell, eps = mu = 1.  Fields q = (Hx, Hy, Hz, Ex, Ey, Ez).

    Upwind flux (the 3D analogue of eq. max2d-numflux, with the factor 1/2):
      flux_H = 1/2 ( n x [E] + alpha (n (n.[H]) - [H]) )
      flux_E = 1/2 (-n x [H] + alpha (n (n.[E]) - [E]) )
    rhs_H = -curl E + LIFT(Fscale flux_H),  rhs_E = curl H + LIFT(Fscale flux_E)."""

    n_fields = 6

    def __init__(self, disc: Discretization3D, alpha: float = 1.0):
        if np.any(disc.eps != 1.0) or np.any(disc.mu != 1.0):
            raise ValueError("3D oracle supports eps = mu = 1 only")
        self.d = disc
        self.alpha = float(alpha)

    def _grad(self, u):
        d, ref = self.d, self.d.ref
        ur, us, ut = _eldot(ref.Dr, u), _eldot(ref.Ds, u), _eldot(ref.Dt, u)
        gx = d.rx[:, None] * ur + d.sx[:, None] * us + d.tx[:, None] * ut
        gy = d.ry[:, None] * ur + d.sy[:, None] * us + d.ty[:, None] * ut
        gz = d.rz[:, None] * ur + d.sz[:, None] * us + d.tz[:, None] * ut
        return gx, gy, gz

    def _curl(self, X, Y, Z):
        Xx, Xy, Xz = self._grad(X)
        Yx, Yy, Yz = self._grad(Y)
        Zx, Zy, Zz = self._grad(Z)
        return Zy - Yz, Xz - Zx, Yx - Xy

    def rhs(self, q: np.ndarray) -> np.ndarray:
        d = self.d
        jumps = [q[f].flat[d.vmapM] - q[f].flat[d.vmapP] for f in range(6)]
        b = d.boundary
        for f in range(3):
            jumps[f][b] = 0.0
        for f in range(3, 6):
            jumps[f][b] = 2.0 * q[f].flat[d.vmapM[b]]
        dH = np.stack(jumps[0:3])
        dE = np.stack(jumps[3:6])
        n = np.stack([d.nx, d.ny, d.nz])
        fH, fE = upwind_flux_3d(n, dH, dE, self.alpha)
        cE = self._curl(q[3], q[4], q[5])
        cH = self._curl(q[0], q[1], q[2])
        L, Fs = d.ref.LIFT, d.Fscale
        out = [-cE[i] + _eldot(L, Fs * fH[i]) for i in range(3)]
        out += [cH[i] + _eldot(L, Fs * fE[i]) for i in range(3)]
        return np.stack(out)

    def energy(self, q: np.ndarray) -> float:
        d, M = self.d, self.d.ref.M
        return 0.5 * sum(float(np.sum(d.J * np.einsum("ki,ij,kj->k", q[f], M, q[f])))
                         for f in range(6))


def cfl_dt(disc, N: int) -> float:
    """Time step from the CFL rule (the paper gives none): dt = (1/2) *
    min LGL spacing(N) * min_k (inradius_k * sqrt(eps_k mu_k)), the inradius
    divided by the local wave speed 1/sqrt(eps mu).  The constant 1/2 keeps
    every eigenvalue of the upwind operator inside the LSRK4 stability region
    for N = 1..8 in 2D and N = 1..4 in 3D (the common 2/3 does not at N = 1)."""
    x = lgl_nodes(N)
    dr = float(x[1] - x[0])
    return 0.5 * dr * float(np.min(disc.inradius() * np.sqrt(disc.eps * disc.mu)))


def steps_for(t_final: float, dt_max: float) -> tuple[int, float]:
    """Nsteps = ceil(t_final/dt_max), dt = t_final/Nsteps."""
    n = int(math.ceil(t_final / dt_max - 1e-12))
    n = max(n, 1)
    return n, t_final / n


def cavity_mode_2d(x, y, t: float, m: int, n: int, eps: float = 1.0, mu: float = 1.0):
    """Closed-form PEC mode of [-1,1]^2 for the 2D TM system:
    Ez = sin(m pi x) sin(n pi y) cos(w t),
    Hx = -(n pi/(mu w)) sin(m pi x) cos(n pi y) sin(w t),
    Hy =  (m pi/(mu w)) cos(m pi x) sin(n pi y) sin(w t),
    w = pi sqrt(m^2+n^2) / sqrt(eps mu)."""
    w = math.pi * math.sqrt(m * m + n * n) / math.sqrt(eps * mu)
    sx, cx = np.sin(m * math.pi * x), np.cos(m * math.pi * x)
    sy, cy = np.sin(n * math.pi * y), np.cos(n * math.pi * y)
    Ez = sx * sy * math.cos(w * t)
    Hx = -(n * math.pi / (mu * w)) * sx * cy * math.sin(w * t)
    Hy = (m * math.pi / (mu * w)) * cx * sy * math.sin(w * t)
    return np.stack([Hx, Hy, Ez])


def cavity_mode_3d(x, y, z, t: float, amp=(1.0, -1.0, 0.0)):
    """Closed-form PEC mode (1,1,1) of [-1,1]^3, eps = mu = 1, A.(1,1,1) = 0:
    E = (Ax cx sy sz, Ay sx cy sz, Az sx sy cz) cos(w t),
    H = -(1/w) curl(E_spatial) sin(w t),  w = pi sqrt(3)."""
    Ax, Ay, Az = amp
    w = math.pi * math.sqrt(3.0)
    p = math.pi
    sx, cx = np.sin(p * x), np.cos(p * x)
    sy, cy = np.sin(p * y), np.cos(p * y)
    sz, cz = np.sin(p * z), np.cos(p * z)
    ct, st = math.cos(w * t), math.sin(w * t)
    Ex = Ax * cx * sy * sz * ct
    Ey = Ay * sx * cy * sz * ct
    Ez = Az * sx * sy * cz * ct
    # curl of the spatial part
    cxE = p * (Az - Ay) * sx * cy * cz
    cyE = p * (Ax - Az) * cx * sy * cz
    czE = p * (Ay - Ax) * cx * cy * sz
    Hx = -cxE * st / w
    Hy = -cyE * st / w
    Hz = -czE * st / w
    return np.stack([Hx, Hy, Hz, Ex, Ey, Ez])
