"""Seeded synthetic workloads (initial data) shaped like the paper's tests.

This module only builds inputs: problem descriptions, initial cell averages
and initial interface point values, plus the exact solutions the paper uses
for its accuracy tables.  It contains none of the scheme's arithmetic and is
shared by the HIP path's tests, the oracle's tests and the benchmark.

Workloads (Sec. 4 of Pan & Xu, arXiv:1412.4489):
  * advection_1d     -- density advection, Sec. 4.1 (Table 1)
  * vortex_2d        -- isentropic vortex, Sec. 4.1 (Table 2), on [0,10]^2
  * sod_1d / blast_1d -- Sec. 4.2
  * sod_2d           -- Sod's problem of Sec. 4.2 in a 2D channel
  * riemann_2d       -- 2D Riemann problems, Sec. 4.3 (cases 1, 2)
  * shock_vortex     -- shock-vortex interaction, Sec. 4.4
  * forward_facing_step -- Sec. 4.6 (a solid step inside the grid)
  * dmr              -- double Mach reflection, Sec. 4.5
  * viscous_shock_tube -- Sec. 4.7 (no-slip adiabatic walls, symmetry line)
  * cavity           -- lid-driven cavity, Sec. 4.8
  * shear_wave / entropy_wave -- linearised Navier-Stokes decay tests
  * batch            -- many independent vortex / Riemann grids of uneven size

Initial point values are the exact initial data at the interface Gauss points
(2D: tangential offsets -+ sqrt(3)/6 of the cell width; 1D: the interface);
where a discontinuity lies on an interface the mean of the two adjacent states
is used.  Cell averages use tensor Gauss-Legendre quadrature (smooth data) or
sub-cell sampling (discontinuous data).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

BC_KINDS = ("periodic", "outflow", "reflect", "noslip_iso", "noslip_adia",
            "inflow", "dmr_bottom", "dmr_top")


@dataclass
class BC:
    kind: str = "periodic"
    state: tuple = (0.0, 0.0, 0.0, 0.0)   # primitive (rho, u, v, p)
    alt: tuple = (0.0, 0.0, 0.0, 0.0)     # second primitive state (DMR pre-shock)
    wall: tuple = (0.0, 0.0, 0.0)         # wall (u, v, T)
    # curvilinear grids: a no-slip wall also turns about the origin at this
    # angular velocity (wall velocity (u - omega y, v + omega x))
    omega: float = 0.0


@dataclass
class Problem:
    dim: int
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    gamma: float = 1.4
    viscous: bool = False
    mu: float = 0.0
    prandtl: float = 1.0
    tau_eps: float = 0.05
    tau_c: float = 1.0
    cfl: float = 0.2
    weno_eps: float = 1e-6
    # C of I(U1) = C h^2 (Sec. 3.1; not printed): large enough that the central
    # polynomial carries smooth regions (the third order of Table 2), small
    # enough that the limited one-sided polynomial carries discontinuities
    weno_c: float = 10.0
    recon_vars: int = 0
    bc: list = field(default_factory=lambda: [BC(), BC(), BC(), BC()])
    # 2D solid step in the lower right corner: cells i >= i0, j < nj
    # ((i0, nj) = (0, 0): none)
    obstacle: tuple = (0, 0)
    # a reconstructed cell polynomial is kept if, at its interface centres,
    # 0: density and pressure are positive (the literal scheme's domain);
    # 1: they also lie within a factor two of the range of the neighbouring
    # averages (else the cell's constant average is used for the step).  The
    # double Mach reflection, the forward-facing step and the viscous shock
    # tube need 1: with 0 they leave the physical states (at 96 x 24 within 70
    # steps; at 240 x 80 by t = 0.52, at 120 x 40 by t = 3.2; at 150 x 75
    # within 3 steps).
    admissibility: int = 0
    t_end: float = 0.0
    name: str = ""
    # 2D curvilinear grid: vertex coordinates [ny+1][nx+1][2] of straight-edged
    # quadrilateral cells (cell (i, j): corners (i, j), (i+1, j), (i+1, j+1),
    # (i, j+1), counter-clockwise); None: the uniform grid of the domain
    mesh: object = None

    @property
    def nvar(self) -> int:
        return self.dim + 2

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.ny if self.dim == 2 else 1.0

    @property
    def ncells(self) -> int:
        return self.nx * self.ny


@dataclass
class State:
    """Host arrays (float64, no ghosts):
    cell[nvar][ny][nx]; fx[ng][nvar][ny][nx+1]; fy[2][nvar][ny+1][nx] (2D)."""
    cell: np.ndarray
    fx: np.ndarray
    fy: np.ndarray

    def copy(self) -> "State":
        return State(self.cell.copy(), self.fx.copy(), self.fy.copy())


GAUSS_OFFSET = math.sqrt(3.0) / 6.0


def cons(gamma, rho, u, v, p, dim=2):
    """Conservative variables from primitive ones (stacked on axis 0)."""
    rho, u, v, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, u, v, p)))
    if dim == 2:
        return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w / 2.0


def _cell_average_2d(fun, prob: Problem, nq=4):
    """Tensor Gauss-Legendre average of fun(x, y) -> (nvar, ...) over each cell."""
    xq, wq = _gl(nq)
    h, k = prob.dx, prob.dy
    xc = prob.x0 + (np.arange(prob.nx) + 0.5) * h
    yc = prob.y0 + (np.arange(prob.ny) + 0.5) * k
    acc = np.zeros((prob.nvar, prob.ny, prob.nx))
    for a in range(nq):
        for b in range(nq):
            X = xc[None, :] + 0.5 * h * xq[a]
            Y = yc[:, None] + 0.5 * k * xq[b]
            X, Y = np.broadcast_arrays(X, Y)
            acc += wq[a] * wq[b] * fun(X, Y)
    return acc


def _quad_average(fun, mesh, nq=4):
    """Average of fun(x, y) -> (nvar, ...) over each straight-edged
    quadrilateral of a vertex grid mesh[ny+1][nx+1][2]: tensor Gauss-Legendre
    on the bilinear map of the corners (exact parametrisation of the cell),
    weighted by its Jacobian."""
    xq, wq = _gl(nq)
    P00, P10 = mesh[:-1, :-1], mesh[:-1, 1:]
    P11, P01 = mesh[1:, 1:], mesh[1:, :-1]
    num, den = 0.0, 0.0
    for a in range(nq):
        for b in range(nq):
            s, t = 0.5 + 0.5 * xq[a], 0.5 + 0.5 * xq[b]
            X = (1 - s) * (1 - t) * P00 + s * (1 - t) * P10 + s * t * P11 + (1 - s) * t * P01
            Xs = (1 - t) * (P10 - P00) + t * (P11 - P01)
            Xt = (1 - s) * (P01 - P00) + s * (P11 - P10)
            J = Xs[..., 0] * Xt[..., 1] - Xs[..., 1] * Xt[..., 0]
            w = wq[a] * wq[b] * J
            num = num + w * fun(X[..., 0], X[..., 1])
            den = den + w
    return num / den


def _quad_face_values(fun, mesh):
    """Values of fun at the two Gauss points of every edge of a vertex grid:
    xi-interfaces (edges along eta) and eta-interfaces (edges along xi), the
    point at -sqrt(3)/6 of the edge first (towards the lower index)."""
    a, b = mesh[:-1, :], mesh[1:, :]      # xi-interfaces [ny][nx+1]
    c, d = mesh[:, :-1], mesh[:, 1:]      # eta-interfaces [ny+1][nx]
    fx = np.stack([fun(*np.moveaxis(0.5 * (a + b) + s * (b - a), -1, 0)) for s in (-GAUSS_OFFSET, GAUSS_OFFSET)])
    fy = np.stack([fun(*np.moveaxis(0.5 * (c + d) + s * (d - c), -1, 0)) for s in (-GAUSS_OFFSET, GAUSS_OFFSET)])
    return np.ascontiguousarray(fx), np.ascontiguousarray(fy)


def polar_mesh(nr, nth, r0=1.0, r1=2.0, th0=-0.5, th1=0.5):
    """Vertices of the grid uniform in (r, theta): xi along r, eta along theta."""
    r = r0 + (r1 - r0) * np.arange(nr + 1) / nr
    th = th0 + (th1 - th0) * np.arange(nth + 1) / nth
    R, TH = np.meshgrid(r, th)
    return np.ascontiguousarray(np.stack([R * np.cos(TH), R * np.sin(TH)], axis=-1))


def mapped_mesh(nx, ny, lx=10.0, ly=10.0, amp=0.0, angle=0.0, shear=0.0):
    """Vertices of [0, lx] x [0, ly] moved by a periodic wave of amplitude amp
    (x += amp lx sin(2 pi x/lx) sin(2 pi y/ly), y likewise), then sheared
    (x += shear y) and turned by angle about the origin.  With amp = 0 the
    cells are parallelograms; the grid stays periodic by translation."""
    x = lx * np.arange(nx + 1) / nx
    y = ly * np.arange(ny + 1) / ny
    X, Y = np.meshgrid(x, y)
    wave = np.sin(2 * math.pi * X / lx) * np.sin(2 * math.pi * Y / ly)
    X, Y = X + amp * lx * wave, Y + amp * ly * wave
    X = X + shear * Y
    c, s = math.cos(angle), math.sin(angle)
    return np.ascontiguousarray(np.stack([c * X - s * Y, s * X + c * Y], axis=-1))


def _face_values_2d(fun, prob: Problem):
    h, k = prob.dx, prob.dy
    xf = prob.x0 + np.arange(prob.nx + 1) * h
    yc = prob.y0 + (np.arange(prob.ny) + 0.5) * k
    xc = prob.x0 + (np.arange(prob.nx) + 0.5) * h
    yf = prob.y0 + np.arange(prob.ny + 1) * k
    fx = np.zeros((2, prob.nvar, prob.ny, prob.nx + 1))
    fy = np.zeros((2, prob.nvar, prob.ny + 1, prob.nx))
    for g, s in enumerate((-GAUSS_OFFSET, GAUSS_OFFSET)):
        X, Y = np.broadcast_arrays(xf[None, :], (yc + s * k)[:, None])
        fx[g] = fun(X, Y)
        X, Y = np.broadcast_arrays((xc + s * h)[None, :], yf[:, None])
        fy[g] = fun(X, Y)
    # on a periodic axis the last interface is the first one: one value
    if prob.bc[0].kind == "periodic":
        fx[..., prob.nx] = fx[..., 0]
    if prob.bc[2].kind == "periodic":
        fy[..., prob.ny, :] = fy[..., 0, :]
    return fx, fy


# --------------------------------------------------------------------------
# 1D
# --------------------------------------------------------------------------

def advection_1d(n=100, cfl=0.5, t_end=2.0, tau_eps=0.0, amp=0.2):
    """Sec. 4.1: rho = 1 + 0.2 sin(pi x), u = 1, p = 1, periodic [0, 2]
    (amp: the amplitude 0.2 of the paper, or another).

    Reading for the smooth accuracy tests: tau = tau_eps dt + |jump| dt with
    tau_eps = 0 (the printed 0.05 dt adds a heat conduction far above the
    errors of Table 1)."""
    g = 1.4
    prob = Problem(dim=1, nx=n, ny=1, x0=0.0, x1=2.0, y0=0.0, y1=1.0, gamma=g,
                   tau_eps=tau_eps, tau_c=1.0, cfl=cfl, t_end=t_end,
                   name=f"advection1d_{n}")
    h = prob.dx
    xl = np.arange(n) * h
    xr = xl + h
    rho_avg = 1.0 + amp * (np.cos(math.pi * xl) - np.cos(math.pi * xr)) / (math.pi * h)
    cell = cons(g, rho_avg, 1.0, 0.0, 1.0, dim=1)
    # rho u and rho E are linear in rho here, so their averages are exact too
    xf = np.arange(n + 1) * h
    fx = cons(g, 1.0 + amp * np.sin(math.pi * xf), 1.0, 0.0, 1.0, dim=1)
    st = State(cell.reshape(3, 1, n), fx.reshape(1, 3, 1, n + 1), np.zeros((2, 3, 2, n)))
    return prob, st


def advection_1d_exact_average(n, t):
    h = 2.0 / n
    xl = np.arange(n) * h - t
    xr = xl + h
    return 1.0 + 0.2 * (np.cos(math.pi * xl) - np.cos(math.pi * xr)) / (math.pi * h)


def _piecewise_1d(n, x0, x1, breaks, states, g, nsub=64):
    """states: list of primitive (rho, u, p) on the intervals split by breaks."""
    h = (x1 - x0) / n
    W = [cons(g, s[0], s[1], 0.0, s[2], dim=1) for s in states]

    def at(x):
        idx = np.searchsorted(np.asarray(breaks), x, side="right")
        return np.stack([W[i] for i in np.atleast_1d(idx)], axis=-1)

    cell = np.zeros((3, n))
    sub = (np.arange(nsub) + 0.5) / nsub
    for i in range(n):
        xs = x0 + (i + sub) * h
        cell[:, i] = at(xs).mean(axis=1)
    xf = x0 + np.arange(n + 1) * h
    fx = at(xf)
    for b in breaks:  # a discontinuity on an interface: mean of both states
        on = np.isclose(xf, b, rtol=0, atol=1e-12 * max(1.0, abs(b)))
        for fi in np.nonzero(on)[0]:
            lo = at(np.array([b - 1e-9 * h]))[:, 0]
            hi = at(np.array([b + 1e-9 * h]))[:, 0]
            fx[:, fi] = 0.5 * (lo + hi)
    return cell, fx


def sod_1d(n=100, t_end=0.2, recon_vars=1):
    """Sec. 4.2 Sod problem on [0, 1]."""
    g = 1.4
    prob = Problem(dim=1, nx=n, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, gamma=g,
                   tau_eps=0.05, tau_c=1.0, cfl=0.2, t_end=t_end, recon_vars=recon_vars,
                   bc=[BC("outflow"), BC("outflow"), BC(), BC()], name=f"sod1d_{n}")
    cell, fx = _piecewise_1d(n, 0.0, 1.0, [0.5], [(1.0, 0.0, 1.0), (0.125, 0.0, 0.1)], g)
    return prob, State(cell.reshape(3, 1, n), fx.reshape(1, 3, 1, n + 1), np.zeros((2, 3, 2, n)))


def viscous_shock_tube_1d(n=600, re=200.0, t_end=0.2, prandtl=0.73, recon_vars=1):
    """The gas of the Sec. 4.7 viscous shock tube along the tube without its
    walls: (rho, u, p) = (120, 0, 120/gamma) for x < 0.5 and (1.2, 0,
    1.2/gamma) beyond on [0, 1], reflecting ends, gamma = 1.4, constant
    mu = 1/Re, Pr 0.73.  On n cells the low-pressure side's cell Knudsen
    number mu/p c / h is about n / (1.2 Re)."""
    g = 1.4
    prob = Problem(dim=1, nx=n, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, gamma=g, viscous=True,
                   mu=1.0 / re, prandtl=prandtl, tau_eps=0.05, tau_c=1.0, cfl=0.2, t_end=t_end,
                   recon_vars=recon_vars, bc=[BC("reflect"), BC("reflect"), BC(), BC()],
                   admissibility=1, name=f"viscous_shock_tube_1d_{n}_re{int(re)}")
    cell, fx = _piecewise_1d(n, 0.0, 1.0, [0.5], [(120.0, 0.0, 120.0 / g), (1.2, 0.0, 1.2 / g)], g)
    return prob, State(cell.reshape(3, 1, n), fx.reshape(1, 3, 1, n + 1), np.zeros((2, 3, 2, n)))


def blast_1d(n=400, t_end=3.8, recon_vars=1):
    """Sec. 4.2 Woodward-Colella blast wave on [0, 100], reflecting ends."""
    g = 1.4
    prob = Problem(dim=1, nx=n, ny=1, x0=0.0, x1=100.0, y0=0.0, y1=1.0, gamma=g,
                   tau_eps=0.05, tau_c=1.0, cfl=0.2, t_end=t_end, recon_vars=recon_vars,
                   bc=[BC("reflect"), BC("reflect"), BC(), BC()], name=f"blast1d_{n}")
    cell, fx = _piecewise_1d(n, 0.0, 100.0, [10.0, 90.0],
                             [(1.0, 0.0, 1000.0), (1.0, 0.0, 0.01), (1.0, 0.0, 100.0)], g)
    return prob, State(cell.reshape(3, 1, n), fx.reshape(1, 3, 1, n + 1), np.zeros((2, 3, 2, n)))


# --------------------------------------------------------------------------
# 2D
# --------------------------------------------------------------------------

def _vortex_fields(X, Y, g, eps, xc, yc):
    dxp, dyp = X - xc, Y - yc
    r2 = dxp * dxp + dyp * dyp
    du = eps / (2 * math.pi) * np.exp(0.5 * (1.0 - r2)) * (-dyp)
    dv = eps / (2 * math.pi) * np.exp(0.5 * (1.0 - r2)) * dxp
    T = 1.0 - (g - 1.0) * eps * eps / (8.0 * g * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (g - 1.0))
    return rho, 1.0 + du, 1.0 + dv, rho * T


def vortex_2d(n=256, t_end=10.0, eps=5.0, cfl=0.2, nq=4, tau_eps=0.0, ny=None):
    """Sec. 4.1 isentropic vortex: mean (rho, u, v, p) = (1, 1, 1, 1), strength
    5, on the periodic square [0, 10]^2 with the vortex centred at (5, 5)."""
    g = 1.4
    ny = n if ny is None else ny
    prob = Problem(dim=2, nx=n, ny=ny, x0=0.0, x1=10.0, y0=0.0, y1=10.0, gamma=g,
                   tau_eps=tau_eps, tau_c=1.0, cfl=cfl, t_end=t_end, name=f"vortex2d_{n}")

    def fun(X, Y):
        return cons(g, *_vortex_fields(X, Y, g, eps, 5.0, 5.0))

    cell = _cell_average_2d(fun, prob, nq=nq)
    fx, fy = _face_values_2d(fun, prob)
    return prob, State(cell, fx, fy)


def vortex_2d_exact_density(prob: Problem, t, eps=5.0, nq=6):
    """Exact cell-average density at time t: the initial vortex carried by the
    mean flow (1, 1); the nearest periodic image of its centre is used."""
    L = prob.x1 - prob.x0
    xc = prob.x0 + ((5.0 + t) - prob.x0) % L
    yc = prob.y0 + ((5.0 + t) - prob.y0) % L

    def fun(X, Y):
        dX = (X - xc + 0.5 * L) % L - 0.5 * L
        dY = (Y - yc + 0.5 * L) % L - 0.5 * L
        rho, *_ = _vortex_fields(dX, dY, prob.gamma, eps, 0.0, 0.0)
        return np.stack([rho] * prob.nvar)

    return _cell_average_2d(fun, prob, nq=nq)[0]


def _piecewise_2d(prob: Problem, state_at, nsub=8):
    """Cell averages by nsub x nsub sub-cell midpoints; point values exact
    (mean of the two sides where the point lies on a discontinuity is left to
    state_at)."""
    h, k = prob.dx, prob.dy
    xc = prob.x0 + (np.arange(prob.nx) + 0.5) * h
    yc = prob.y0 + (np.arange(prob.ny) + 0.5) * k
    sub = (np.arange(nsub) + 0.5) / nsub - 0.5
    acc = np.zeros((prob.nvar, prob.ny, prob.nx))
    for a in sub:
        for b in sub:
            X, Y = np.broadcast_arrays(xc[None, :] + a * h, yc[:, None] + b * k)
            acc += state_at(X, Y)
    cell = acc / (nsub * nsub)
    fx, fy = _face_values_2d(state_at, prob)
    return cell, fx, fy


RIEMANN_CASES = {
    # (rho, u, v, p) in quadrants NE, NW, SW, SE (Sec. 4.3)
    1: [(0.5313, 0.0, 0.0, 0.4), (1.0, 0.7276, 0.0, 1.0), (0.8, 0.0, 0.0, 1.0), (1.0, 0.0, 0.7276, 1.0)],
    2: [(1.0, 0.75, -0.5, 1.0), (2.0, 0.75, 0.5, 1.0), (1.0, -0.75, 0.5, 1.0), (3.0, -0.75, -0.5, 1.0)],
}


def riemann_2d(case=1, n=200, t_end=0.2, nx=None, ny=None, recon_vars=0):
    """Sec. 4.3: quadrant Riemann problems on [0, 1]^2, non-reflecting
    (zero-gradient) boundaries."""
    g = 1.4
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    prob = Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=1.0, gamma=g,
                   tau_eps=0.05, tau_c=1.0, cfl=0.2, t_end=t_end, recon_vars=recon_vars,
                   bc=[BC("outflow") for _ in range(4)], name=f"riemann{case}_{nx}x{ny}")
    Q = np.stack([cons(g, *s) for s in RIEMANN_CASES[case]])

    def raw(X, Y):
        east, north = X > 0.5, Y > 0.5
        quad = np.where(north, np.where(east, 0, 1), np.where(east, 3, 2))
        return np.moveaxis(Q[quad], -1, 0)

    def state_at(X, Y):
        # mean over four tiny offsets: the exact state off the discontinuity
        # lines, the mean of the adjacent states on them
        d = 1e-9
        return 0.25 * sum(raw(X + sx, Y + sy) for sx in (-d, d) for sy in (-d, d))

    cell, fx, fy = _piecewise_2d(prob, state_at)
    return prob, State(cell, fx, fy)


def sod_2d(n=100, m=4, axis=0, t_end=0.2, recon_vars=1):
    """Sod's problem of Sec. 4.2 in a 2D channel: the tube along x (axis 0,
    n x m cells on [0, 1] x [0, m/n]) or along y (axis 1), zero-gradient ends
    and periodic across the channel."""
    g = 1.4
    w = m / n
    if axis == 0:
        nx, ny, x1, y1 = n, m, 1.0, w
        bc = [BC("outflow"), BC("outflow"), BC(), BC()]
    else:
        nx, ny, x1, y1 = m, n, w, 1.0
        bc = [BC(), BC(), BC("outflow"), BC("outflow")]
    prob = Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=x1, y0=0.0, y1=y1, gamma=g,
                   tau_eps=0.05, tau_c=1.0, cfl=0.2, t_end=t_end, recon_vars=recon_vars, bc=bc,
                   name=f"sod2d_{'xy'[axis]}_{n}")
    left, right = cons(g, 1.0, 0.0, 0.0, 1.0), cons(g, 0.125, 0.0, 0.0, 0.1)

    def state_at(X, Y):
        s = X if axis == 0 else Y
        d = 1e-9
        lo = np.where(s - d < 0.5, 1.0, 0.0)[None]
        hi = np.where(s + d < 0.5, 1.0, 0.0)[None]
        wl = 0.5 * (lo + hi)
        return wl * left.reshape(4, *([1] * X.ndim)) + (1.0 - wl) * right.reshape(4, *([1] * X.ndim))

    cell, fx, fy = _piecewise_2d(prob, state_at)
    return prob, State(cell, fx, fy)


SHOCK_VORTEX_MACH = 1.1


def shock_vortex(nx=201, ny=101, t_end=0.8, kappa=0.3, mu=0.204, rc=0.05, recon_vars=1):
    """Sec. 4.4 shock-vortex interaction on [0, 2] x [0, 1]: a stationary
    Mach 1.1 normal shock at x = 0.5, upstream state (Ma^2, sqrt(gamma), 0, 1),
    downstream state from the Rankine-Hugoniot relations, and an isentropic
    vortex centred at (0.25, 0.5) on the upstream flow (velocity perturbation
    kappa eta exp(mu (1 - eta^2)) (sin theta, -cos theta), temperature
    perturbation -(gamma - 1) kappa^2 / (4 mu gamma) exp(2 mu (1 - eta^2)),
    entropy unchanged, eta = r / rc).  Reflecting top and bottom, the upstream
    state flowing in on the left, zero-gradient outflow on the right."""
    g = 1.4
    M = SHOCK_VORTEX_MACH
    up = (M * M, math.sqrt(g), 0.0, 1.0)
    rr = (g + 1.0) * M * M / ((g - 1.0) * M * M + 2.0)
    pr = 1.0 + 2.0 * g / (g + 1.0) * (M * M - 1.0)
    down = (up[0] * rr, up[1] / rr, 0.0, up[3] * pr)
    bc = [BC("inflow", state=up), BC("outflow"), BC("reflect"), BC("reflect")]
    prob = Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=2.0, y0=0.0, y1=1.0, gamma=g,
                   tau_eps=0.05, tau_c=1.0, cfl=0.2, t_end=t_end, recon_vars=recon_vars, bc=bc,
                   name=f"shock_vortex_{nx}x{ny}")
    T0 = up[3] / up[0]
    S0 = up[3] / up[0] ** g

    def state_at(X, Y):
        dx, dy = X - 0.25, Y - 0.5
        r = np.hypot(dx, dy)
        eta = r / rc
        e = np.exp(mu * (1.0 - eta * eta))
        # (sin theta, -cos theta) r = (dy, -dx)
        amp = np.where(r > 0.0, kappa * eta * e / np.where(r > 0.0, r, 1.0), 0.0)
        T = T0 - (g - 1.0) * kappa * kappa / (4.0 * mu * g) * e * e
        rho = (T / S0) ** (1.0 / (g - 1.0))
        upstream = cons(g, rho, up[1] + amp * dy, amp * -dx, rho * T)
        downstream = cons(g, *[np.full(X.shape, q) for q in down])
        d = 1e-9
        wl = 0.5 * (np.where(X - d < 0.5, 1.0, 0.0) + np.where(X + d < 0.5, 1.0, 0.0))[None]
        return wl * upstream + (1.0 - wl) * downstream

    cell, fx, fy = _piecewise_2d(prob, state_at)
    return prob, State(cell, fx, fy)


def forward_facing_step(nx=120, ny=40, t_end=4.0, recon_vars=1):
    """Sec. 4.6 forward-facing step: the tunnel [0, 3] x [0, 1] with a solid
    step from x = 0.6 to the exit of height 0.2 (cells i >= 0.2 nx,
    j < 0.2 ny), a Mach 3 flow (rho, u, v, p) = (1.4, 3, 0, 1) everywhere at
    t = 0 and flowing in on the left, outflow on the right, slip walls on
    the tunnel's walls and the step."""
    g = 1.4
    if nx % 5 or ny % 5:
        raise ValueError("nx and ny must be multiples of 5 (the step on cell edges)")
    state = (1.4, 3.0, 0.0, 1.0)
    bc = [BC("inflow", state=state), BC("outflow"), BC("reflect"), BC("reflect")]
    prob = Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=3.0, y0=0.0, y1=1.0, gamma=g,
                   tau_eps=0.05, tau_c=1.0, cfl=0.2, t_end=t_end, recon_vars=recon_vars, bc=bc,
                   obstacle=(nx // 5, ny // 5), admissibility=1, name=f"forward_facing_step_{nx}x{ny}")
    q = cons(g, *state)
    cell = np.broadcast_to(q[:, None, None], (4, ny, nx)).copy()
    fx = np.broadcast_to(q[None, :, None, None], (2, 4, ny, nx + 1)).copy()
    fy = np.broadcast_to(q[None, :, None, None], (2, 4, ny + 1, nx)).copy()
    return prob, State(cell, fx, fy)


DMR_POST = (8.0, 4.125 * math.sqrt(3.0), -4.125, 116.5)
DMR_PRE = (1.4, 0.0, 0.0, 1.0)


def dmr(nx=1920, ny=480, t_end=0.2, recon_vars=0):
    """Sec. 4.5 double Mach reflection on [0, 4] x [0, 1]: a Mach 10 shock
    through (1/6, 0) at 60 degrees; post-shock inflow at the left edge and on
    the bottom for x < 1/6, slip wall beyond, exact shock motion on top,
    zero-gradient outflow on the right."""
    g = 1.4
    bc = [BC("inflow", state=DMR_POST), BC("outflow"),
          BC("dmr_bottom", state=DMR_POST), BC("dmr_top", state=DMR_POST, alt=DMR_PRE)]
    prob = Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=4.0, y0=0.0, y1=1.0, gamma=g,
                   tau_eps=0.05, tau_c=1.0, cfl=0.2, t_end=t_end, bc=bc, recon_vars=recon_vars,
                   admissibility=1, name=f"dmr_{nx}x{ny}")
    post, pre = cons(g, *DMR_POST), cons(g, *DMR_PRE)
    s3 = math.sqrt(3.0)

    def state_at(X, Y):
        behind = X < 1.0 / 6.0 + Y / s3
        out = np.where(behind[None], post.reshape(4, *([1] * X.ndim)), pre.reshape(4, *([1] * X.ndim)))
        return out

    cell, fx, fy = _piecewise_2d(prob, state_at)
    return prob, State(cell, fx, fy)


def cavity(n=512, re=1000.0, mach=0.15, prandtl=0.72, gamma=5.0 / 3.0, lid_transits=20.0):
    """Sec. 4.8 lid-driven cavity on [0, 1]^2: gas at rest (rho = 1, T = 1),
    isothermal no-slip walls at T = 1, lid velocity Ma * sqrt(gamma) on top;
    constant mu = U_lid / Re."""
    g = gamma
    ulid = mach * math.sqrt(g)
    mu = ulid / re
    bc = [BC("noslip_iso", wall=(0.0, 0.0, 1.0)), BC("noslip_iso", wall=(0.0, 0.0, 1.0)),
          BC("noslip_iso", wall=(0.0, 0.0, 1.0)), BC("noslip_iso", wall=(ulid, 0.0, 1.0))]
    prob = Problem(dim=2, nx=n, ny=n, x0=0.0, x1=1.0, y0=0.0, y1=1.0, gamma=g, viscous=True,
                   mu=mu, prandtl=prandtl, tau_eps=0.0, tau_c=1.0, cfl=0.2,
                   t_end=lid_transits / ulid, bc=bc, name=f"cavity_{n}_re{int(re)}")
    cell = np.zeros((4, n, n))
    cell[:] = cons(g, 1.0, 0.0, 0.0, 1.0)[:, None, None]
    fx = np.broadcast_to(cell[:, :, :1], (4, n, n + 1))[None].repeat(2, axis=0).copy()
    fy = np.broadcast_to(cell[:, :1, :], (4, n + 1, n))[None].repeat(2, axis=0).copy()
    return prob, State(cell, fx, fy)


def viscous_shock_tube(nx=300, ny=150, re=200.0, t_end=1.0, prandtl=0.73, recon_vars=1):
    """Sec. 4.7 viscous shock tube on [0, 1] x [0, 0.5]: gas at rest,
    (rho, p) = (120, 120/gamma) for x < 0.5 and (1.2, 1.2/gamma) beyond,
    gamma = 1.4; no-slip adiabatic walls on the left, right and bottom, the
    symmetry line (a slip wall) on top; constant mu = 1/Re, Pr = 0.73."""
    g = 1.4
    wall = BC("noslip_adia", wall=(0.0, 0.0, 0.0))
    bc = [wall, BC("noslip_adia", wall=(0.0, 0.0, 0.0)), BC("noslip_adia", wall=(0.0, 0.0, 0.0)),
          BC("reflect")]
    prob = Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=0.5, gamma=g, viscous=True,
                   mu=1.0 / re, prandtl=prandtl, tau_eps=0.05, tau_c=1.0, cfl=0.2, t_end=t_end,
                   recon_vars=recon_vars, bc=bc, admissibility=1,
                   name=f"viscous_shock_tube_{nx}x{ny}_re{int(re)}")
    left, right = cons(g, 120.0, 0.0, 0.0, 120.0 / g), cons(g, 1.2, 0.0, 0.0, 1.2 / g)

    def state_at(X, Y):
        d = 1e-9
        wl = 0.5 * (np.where(X - d < 0.5, 1.0, 0.0) + np.where(X + d < 0.5, 1.0, 0.0))[None]
        return wl * left.reshape(4, *([1] * X.ndim)) + (1.0 - wl) * right.reshape(4, *([1] * X.ndim))

    cell, fx, fy = _piecewise_2d(prob, state_at)
    return prob, State(cell, fx, fy)


def shear_wave(n=32, m=4, amp=1e-3, mu=0.01, prandtl=1.0, gamma=1.4):
    """Linearised Navier-Stokes test: rho = p = 1 at rest except the
    transverse velocity v = amp sin(2 pi x) on the periodic [0, 1] x [0, m/n];
    its amplitude decays as exp(-(mu / rho) (2 pi)^2 t)."""
    prob = Problem(dim=2, nx=n, ny=m, x0=0.0, x1=1.0, y0=0.0, y1=m / n, gamma=gamma, viscous=True,
                   mu=mu, prandtl=prandtl, tau_eps=0.0, tau_c=1.0, cfl=0.2, name=f"shear_wave_{n}")

    def fun(X, Y):
        return cons(gamma, np.ones_like(X), np.zeros_like(X), amp * np.sin(2 * np.pi * X), np.ones_like(X))

    cell = _cell_average_2d(fun, prob, nq=6)
    fx, fy = _face_values_2d(fun, prob)
    return prob, State(cell, fx, fy)


def entropy_wave(n=32, m=4, amp=1e-3, mu=0.01, prandtl=0.72, gamma=1.4):
    """Linearised Navier-Stokes test: at rest under the uniform pressure 1,
    temperature T = 1 + amp sin(2 pi x) (rho = 1/T) on the periodic
    [0, 1] x [0, m/n]; heat conduction makes the temperature amplitude decay
    as exp(-kappa (2 pi)^2 t / (rho c_p)) with kappa = c_p mu / Pr, i.e. at
    the rate mu (2 pi)^2 / (rho Pr)."""
    prob = Problem(dim=2, nx=n, ny=m, x0=0.0, x1=1.0, y0=0.0, y1=m / n, gamma=gamma, viscous=True,
                   mu=mu, prandtl=prandtl, tau_eps=0.0, tau_c=1.0, cfl=0.2, name=f"entropy_wave_{n}")

    def fun(X, Y):
        T = 1.0 + amp * np.sin(2 * np.pi * X)
        return cons(gamma, 1.0 / T, np.zeros_like(X), np.zeros_like(X), np.ones_like(X))

    cell = _cell_average_2d(fun, prob, nq=6)
    fx, fy = _face_values_2d(fun, prob)
    return prob, State(cell, fx, fy)


BATCH_SIZES = (64, 96, 128, 192, 256, 384)


def batch(n_problems=96, seed=14124489, sizes=BATCH_SIZES):
    """Many independent 2D grids of uneven size advanced together: the
    isentropic vortex of Sec. 4.1 (half of the problems, periodic [0, 10]^2)
    and the quadrant Riemann problems 1 and 2 of Sec. 4.3 (a quarter each,
    zero-gradient boundaries on [0, 1]^2), on n x n cells with n drawn
    uniformly from `sizes`.  Every problem draws Euler or Navier-Stokes
    (half each) and Re log-uniform in [100, 5000] (U_ref = 1, rho_ref = 1,
    L = the vortex's unit core radius, constant mu, Pr 0.72); the draw makes
    the vortex problems viscous, while the Riemann problems stay the
    inviscid tests of Sec. 4.3: from their sharp initial jumps, tau |grad W|
    of the Navier-Stokes distribution is of order one at Re of a few hundred
    on 96^2 - 192^2 cells, outside its Chapman-Enskog range, and the scheme
    leaves the physical states within the first steps (in the oracle as on
    the GPU).  Collision time: Euler vortex tau_eps = 0 (smooth data),
    Riemann tau_eps = 0.05, Navier-Stokes mu/p plus the jump term (Sec. 4).
    Returns a list of (Problem, State)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_problems):
        r = rng.uniform()
        kind = "vortex" if r < 0.5 else ("riemann1" if r < 0.75 else "riemann2")
        n = int(rng.choice(np.asarray(sizes)))
        viscous = bool(rng.uniform() < 0.5)
        re = float(math.exp(rng.uniform(math.log(100.0), math.log(5000.0))))
        if kind == "vortex":
            prob, st = vortex_2d(n)
        else:
            prob, st = riemann_2d(1 if kind == "riemann1" else 2, n=n)
        if viscous and kind == "vortex":
            prob = replace(prob, viscous=True, mu=1.0 / re, prandtl=0.72, tau_eps=0.0)
        prob = replace(prob, name=f"batch{k}_{prob.name}_{'ns' if prob.viscous else 'euler'}")
        out.append((prob, st))
    return out


def uniform_2d(nx=16, ny=12, state=(1.3, 0.4, -0.7, 2.1), gamma=1.4, bc="periodic", **kw):
    """Free stream: one uniform state everywhere."""
    prob = Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=0.75, gamma=gamma,
                   bc=[BC(bc) for _ in range(4)], name="uniform", **kw)
    q = cons(gamma, *state)
    cell = np.broadcast_to(q[:, None, None], (4, ny, nx)).copy()
    fx = np.broadcast_to(q[None, :, None, None], (2, 4, ny, nx + 1)).copy()
    fy = np.broadcast_to(q[None, :, None, None], (2, 4, ny + 1, nx)).copy()
    return prob, State(cell, fx, fy)


def smooth_periodic_2d(nx=24, ny=20, seed=0, amp=0.1, gamma=1.4, viscous=False, mu=0.0,
                       prandtl=1.0, tau_eps=0.05, lx=1.0, ly=1.0):
    """A seeded smooth periodic flow: low-mode Fourier perturbations of a
    uniform state in rho, u, v, p (for parity and conservation tests)."""
    rng = np.random.default_rng(seed)
    prob = Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=lx, y0=0.0, y1=ly, gamma=gamma,
                   viscous=viscous, mu=mu, prandtl=prandtl, tau_eps=tau_eps,
                   name=f"smooth_{nx}x{ny}_s{seed}")
    base = np.array([1.0, 0.3, -0.2, 1.0])
    modes = []
    for q in range(4):
        for _ in range(3):
            kx, ky = rng.integers(0, 3, size=2)
            a, ph = rng.uniform(-amp, amp), rng.uniform(0, 2 * math.pi)
            modes.append((q, kx, ky, a, ph))

    def fun(X, Y):
        prim = [np.full(X.shape, base[q]) for q in range(4)]
        for q, kx, ky, a, ph in modes:
            prim[q] = prim[q] + a * np.sin(2 * math.pi * (kx * X / lx + ky * Y / ly) + ph)
        return cons(gamma, *prim)

    cell = _cell_average_2d(fun, prob, nq=4)
    fx, fy = _face_values_2d(fun, prob)
    return prob, State(cell, fx, fy)


def random_perturbed_2d(nx=24, ny=20, seed=0, amp=0.2, gamma=1.4, bc="periodic", **kw):
    """Seeded rough data: a uniform state with independent random cell and
    point-value perturbations (exercises every limiter branch)."""
    rng = np.random.default_rng(seed)
    prob = Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=ny / nx,
                   gamma=gamma, bc=[BC(bc) for _ in range(4)], name=f"rough_{nx}x{ny}_s{seed}", **kw)

    def draw(shape):
        rho = 1.0 + amp * rng.uniform(-1, 1, shape)
        u = 0.5 * amp * rng.uniform(-1, 1, shape) + 0.2
        v = 0.5 * amp * rng.uniform(-1, 1, shape) - 0.1
        p = 1.0 + amp * rng.uniform(-1, 1, shape)
        return cons(gamma, rho, u, v, p)

    cell = draw((ny, nx))
    fx = np.stack([draw((ny, nx + 1)), draw((ny, nx + 1))], axis=0)
    fy = np.stack([draw((ny + 1, nx)), draw((ny + 1, nx))], axis=0)
    if bc == "periodic":  # the first and last interfaces are the same interface
        fx[..., nx] = fx[..., 0]
        fy[..., ny, :] = fy[..., 0, :]
    return prob, State(np.ascontiguousarray(cell), np.ascontiguousarray(fx), np.ascontiguousarray(fy))


# --------------------------------------------------------------------------
# curvilinear grids (the extension the remark closing Sec. 3.3 points to;
# the polar cavity of Sec. 4.8)
# --------------------------------------------------------------------------

def _mesh_problem(mesh, **kw):
    ny, nx = mesh.shape[0] - 1, mesh.shape[1] - 1
    lo, hi = mesh.reshape(-1, 2).min(axis=0), mesh.reshape(-1, 2).max(axis=0)
    return Problem(dim=2, nx=nx, ny=ny, x0=float(lo[0]), x1=float(hi[0]), y0=float(lo[1]), y1=float(hi[1]),
                   mesh=mesh, **kw)


def _mesh_state(prob, fun, nq=4):
    cell = np.ascontiguousarray(_quad_average(fun, prob.mesh, nq=nq))
    fx, fy = _quad_face_values(fun, prob.mesh)
    if prob.bc[0].kind == "periodic":
        fx[..., prob.nx] = fx[..., 0]
    if prob.bc[2].kind == "periodic":
        fy[..., prob.ny, :] = fy[..., 0, :]
    return State(cell, np.ascontiguousarray(fx), np.ascontiguousarray(fy))


def _lattice_vortex(X, Y, g, eps, centre, A, B, mean):
    """the isentropic vortex of Sec. 4.1 (strength eps, unit core) centred at
    the periodic image of `centre` nearest to (X, Y) on the lattice spanned
    by A and B, carried by the mean flow `mean` (rho = p = 1 at infinity)"""
    M = np.array([[A[0], B[0]], [A[1], B[1]]])
    Mi = np.linalg.inv(M)
    dX, dY = X - centre[0], Y - centre[1]
    a = Mi[0, 0] * dX + Mi[0, 1] * dY
    b = Mi[1, 0] * dX + Mi[1, 1] * dY
    a -= np.floor(a + 0.5)
    b -= np.floor(b + 0.5)
    dxp = M[0, 0] * a + M[0, 1] * b
    dyp = M[1, 0] * a + M[1, 1] * b
    r2 = dxp * dxp + dyp * dyp
    du = eps / (2 * math.pi) * np.exp(0.5 * (1.0 - r2)) * (-dyp)
    dv = eps / (2 * math.pi) * np.exp(0.5 * (1.0 - r2)) * dxp
    T = 1.0 - (g - 1.0) * eps * eps / (8.0 * g * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (g - 1.0))
    return rho, mean[0] + du, mean[1] + dv, rho * T


def vortex_mapped(n=64, amp=0.0, angle=0.0, shear=0.0, t_end=10.0, eps=5.0, cfl=0.2, nq=4):
    """The isentropic vortex of Sec. 4.1 on a curvilinear periodic grid:
    [0, 10]^2 with n x n cells, waved (amp), sheared and turned by `angle`
    (mapped_mesh); the mean flow (1, 1) and the vortex centre (5, 5) are
    carried by the same shear and turn, so with amp = shear = 0 the problem is
    the Cartesian vortex turned as a whole."""
    g = 1.4
    mesh = mapped_mesh(n, n, 10.0, 10.0, amp=amp, angle=angle, shear=shear)
    c, s_ = math.cos(angle), math.sin(angle)

    def turn(x, y):
        x = x + shear * y
        return (c * x - s_ * y, s_ * x + c * y)

    A, B, centre = turn(10.0, 0.0), turn(0.0, 10.0), turn(5.0, 5.0)
    mean = (c - s_, s_ + c) if shear == 0.0 else turn(1.0, 1.0)
    prob = _mesh_problem(mesh, gamma=g, tau_eps=0.0, tau_c=1.0, cfl=cfl, t_end=t_end,
                         name=f"vortex_mapped_{n}")
    prob.vortex = dict(eps=eps, centre=centre, A=A, B=B, mean=mean)

    def fun(X, Y):
        return cons(g, *_lattice_vortex(X, Y, g, eps, centre, A, B, mean))

    return prob, _mesh_state(prob, fun, nq=nq)


def vortex_mapped_exact_density(prob, t, nq=6):
    """exact cell-average density of vortex_mapped at time t"""
    v = prob.vortex
    centre = (v["centre"][0] + v["mean"][0] * t, v["centre"][1] + v["mean"][1] * t)

    def fun(X, Y):
        return _lattice_vortex(X, Y, prob.gamma, v["eps"], centre, v["A"], v["B"], v["mean"])[0][None]

    return _quad_average(fun, prob.mesh, nq=nq)[0]


def uniform_mesh(mesh, state=(1.3, 0.4, -0.7, 2.1), gamma=1.4, bc="periodic", **kw):
    """Free stream on a curvilinear grid (periodic, or the state flowing in on
    every side)."""
    prob = _mesh_problem(mesh, gamma=gamma, name="uniform_mesh", **kw)
    prob.bc = [BC(bc, state=state) for _ in range(4)]
    q = cons(gamma, *state)
    return prob, _mesh_state(prob, lambda X, Y: np.broadcast_to(q.reshape(4, *([1] * X.ndim)), (4,) + X.shape).copy())


def solid_rotation(n=32, omega=0.5, viscous=False, mu=1e-3, prandtl=0.72, gamma=5.0 / 3.0, t_end=1.0,
                   cfl=0.2):
    """Gas turning as a solid body, u = omega (-y, x), at the uniform
    temperature 1, in the annulus 1 < r < 2 (the radii of the polar cavity of
    Sec. 4.8) with n cells across and 4n around (periodic in theta): density
    rho = exp(omega^2 (r^2 - 1)/2) holds the radial pressure gradient.  Both
    walls are isothermal (T = 1) and turn with the gas, so this state is
    steady for the Euler and the Navier-Stokes equations (no strain, no heat
    flux)."""
    mesh = polar_mesh(n, 4 * n, th0=-math.pi, th1=math.pi)
    mesh[-1] = mesh[0]  # the seam: the same vertices
    bc = [BC("noslip_iso", wall=(0.0, 0.0, 1.0), omega=omega) for _ in range(2)] + [BC("periodic"), BC("periodic")]
    prob = _mesh_problem(mesh, gamma=gamma, viscous=viscous, mu=mu if viscous else 0.0,
                         prandtl=prandtl if viscous else 1.0, tau_eps=0.05, tau_c=1.0, cfl=cfl, t_end=t_end,
                         bc=bc, name=f"solid_rotation_{n}")
    prob.rotation = omega

    def fun(X, Y):
        rho = np.exp(0.5 * omega * omega * (X * X + Y * Y - 1.0))
        return cons(gamma, rho, -omega * Y, omega * X, rho)

    return prob, _mesh_state(prob, fun, nq=6)


def solid_rotation_exact(prob, nq=6):
    """exact cell averages of solid_rotation (steady)"""
    w, g = prob.rotation, prob.gamma

    def fun(X, Y):
        rho = np.exp(0.5 * w * w * (X * X + Y * Y - 1.0))
        return cons(g, rho, -w * Y, w * X, rho)

    return _quad_average(fun, prob.mesh, nq=nq)


def polar_cavity(n=65, re=350.0, mach=0.15, prandtl=0.72, gamma=5.0 / 3.0, turns=20.0):
    """Sec. 4.8 polar cavity: (r, theta) in [1, 2] x [-0.5, 0.5], uniform in r
    and theta ("65 x 65 mesh points" read as cells, like the square cavity),
    gas at rest (rho = 1, T = 1), isothermal no-slip walls at T = 1; the inner
    wall r = 1 turns anticlockwise at the speed U_i = Ma sqrt(gamma) (angular
    velocity U_i / R_i, R_i = 1); constant mu = U_i R_i / Re.  The end time
    is `turns` passages of the inner wall's speed across the unit gap."""
    ui = mach * math.sqrt(gamma)
    mesh = polar_mesh(n, n)
    wall = (0.0, 0.0, 1.0)
    bc = [BC("noslip_iso", wall=wall, omega=ui), BC("noslip_iso", wall=wall),
          BC("noslip_iso", wall=wall), BC("noslip_iso", wall=wall)]
    prob = _mesh_problem(mesh, gamma=gamma, viscous=True, mu=ui / re, prandtl=prandtl, tau_eps=0.0, tau_c=1.0,
                         cfl=0.2, t_end=turns / ui, bc=bc, name=f"polar_cavity_{n}_re{int(re)}")
    q = cons(gamma, 1.0, 0.0, 0.0, 1.0)
    return prob, _mesh_state(prob, lambda X, Y: np.broadcast_to(q.reshape(4, *([1] * X.ndim)), (4,) + X.shape).copy())


def mirror_extension(prob, st, axis):
    """the problem doubled across its low edge along `axis` (0: x, 1: y) with
    the mirror image of the data there (normal momentum negated, Gauss points
    along the edge's direction swapped)"""
    m = 1 + axis  # normal momentum component
    if axis == 1:
        D = replace(prob, ny=2 * prob.ny, y0=prob.y0 - (prob.y1 - prob.y0))
        c = np.concatenate([st.cell[:, ::-1, :], st.cell], axis=1)
        fx = np.concatenate([st.fx[::-1, :, ::-1, :], st.fx], axis=2)
        fy = np.concatenate([st.fy[:, :, ::-1, :][:, :, :-1, :], st.fy], axis=2)
        c[m, :prob.ny] *= -1
        fx[:, m, :prob.ny] *= -1
        fy[:, m, :prob.ny] *= -1
    else:
        D = replace(prob, nx=2 * prob.nx, x0=prob.x0 - (prob.x1 - prob.x0))
        c = np.concatenate([st.cell[:, :, ::-1], st.cell], axis=2)
        fx = np.concatenate([st.fx[:, :, :, ::-1][:, :, :, :-1], st.fx], axis=3)
        fy = np.concatenate([st.fy[::-1, :, :, ::-1], st.fy], axis=3)
        c[m, :, :prob.nx] *= -1
        fx[:, m, :, :prob.nx] *= -1
        fy[:, m, :, :prob.nx] *= -1
    return D, State(np.ascontiguousarray(c), np.ascontiguousarray(fx), np.ascontiguousarray(fy))


def state_for(prob: Problem, cell, fx, fy=None) -> State:
    if fy is None:
        fy = np.zeros((2, prob.nvar, prob.ny + 1, prob.nx))
    return State(cell, fx, fy)
