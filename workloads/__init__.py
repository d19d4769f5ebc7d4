"""Seeded synthetic workloads for the AZ RBF solver.

This module describes *problems*, not the method: domains (membership
predicates and boundary curves), right-hand-side functions, boundary-point
placement, test-point sets and the served request stream.  It holds none of
the solver's arithmetic (no grids, kernels, spectra or linear algebra) and is
the only code shared by the CPU oracle and the GPU path.

Every problem follows the paper's setting: Gaussian RBF centres on a regular
grid over the bounding box [-T, T) (section 2.2, eq. set_centers), collocation
points taken from an s-times finer grid inside the domain (eq. set_X,
eq. set_X_2d), and for boundary value problems weakly imposed Dirichlet data at
points on the boundary (section 6.2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

__all__ = [
    "Domain", "interval", "disk", "star", "ellipse", "box", "flower", "with_hole", "shape_parameter_eh",
    "Problem", "trig_sum_1d", "trig_sum_2d",
    "config_c1", "config_c1a", "config_c2", "config_c3", "config_c3a",
    "config_c4", "config_ellipse", "config_flower", "family_1d", "served_stream", "test_points",
]


# --------------------------------------------------------------------------
# Domains
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Domain:
    """A domain inside the bounding box.

    ``contains`` maps coordinate arrays to a boolean mask.  Membership is
    inclusive (points on the boundary belong to the domain).  For 2D domains
    that are star-shaped about the origin, ``radius`` gives the boundary as
    r(theta) and ``dradius`` its derivative; they define boundary points.
    ``holes`` lists circles (cx, cy, r) cut out of a 2D domain (a multiply
    connected domain); their circles are part of the boundary.
    """
    name: str
    dim: int
    contains: Callable[..., np.ndarray]
    bounds: Optional[tuple] = None
    radius: Optional[Callable[[np.ndarray], np.ndarray]] = None
    dradius: Optional[Callable[[np.ndarray], np.ndarray]] = None
    area: Optional[float] = None
    holes: tuple = ()


def interval(a: float, b: float) -> Domain:
    return Domain(f"interval[{a},{b}]", 1,
                  lambda x: (x >= a) & (x <= b), bounds=(a, b), area=b - a)


def box(T: float = 1.0, dim: int = 1, Ty: Optional[float] = None) -> Domain:
    """The whole periodic box (the periodic problems of sections 3.1 and 5.1)."""
    if dim == 2:
        ty = T if Ty is None else Ty
        return Domain("box", 2, lambda x, y: np.ones(np.shape(x), dtype=bool),
                      bounds=(-T, T), area=4 * T * ty)
    return Domain("box", 1, lambda x: np.ones(np.shape(x), dtype=bool),
                  bounds=(-T, T), area=2 * T)


def shape_parameter_eh(tau0: float) -> float:
    """eps*h of the paper's shape-parameter rule (eq. constant_shapeparam):
    pi / sqrt(2 log(1 + tau0^-2)), which makes the smallest entry of the
    kernel's symbol about tau0 (Lemma 4.3)."""
    return math.pi / math.sqrt(2.0 * math.log1p(tau0 ** -2))


def disk(R: float) -> Domain:
    return Domain(f"disk(R={R})", 2,
                  lambda x, y: x * x + y * y <= R * R,
                  radius=lambda t: np.full(np.shape(t), R, dtype=np.float64),
                  dradius=lambda t: np.zeros(np.shape(t), dtype=np.float64),
                  area=math.pi * R * R)


def ellipse(a: float, b: float) -> Domain:
    """Ellipse x^2/a^2 + y^2/b^2 <= 1 (the domain of section 5.4's
    non-periodic experiment is a = 1, b = 1/2)."""
    def radius(t):
        return 1.0 / np.sqrt((np.cos(t) / a) ** 2 + (np.sin(t) / b) ** 2)

    def dradius(t):
        r = radius(t)
        return -r ** 3 * np.sin(t) * np.cos(t) * (1.0 / (b * b) - 1.0 / (a * a))
    return Domain(f"ellipse(a={a},b={b})", 2, lambda x, y: (x / a) ** 2 + (y / b) ** 2 <= 1.0,
                  radius=radius, dradius=dradius, area=math.pi * a * b)


def star(R: float, amp: float = 0.1, petals: int = 5) -> Domain:
    """Star domain r(theta) = R + amp*cos(petals*theta)."""
    def contains(x, y):
        return np.sqrt(x * x + y * y) <= R + amp * np.cos(petals * np.arctan2(y, x))
    return Domain(f"star(R={R},a={amp},p={petals})", 2, contains,
                  radius=lambda t: R + amp * np.cos(petals * t),
                  dradius=lambda t: -amp * petals * np.sin(petals * t),
                  area=math.pi * (R * R + 0.5 * amp * amp))


def with_hole(dom: Domain, cx: float, cy: float, r: float) -> Domain:
    """``dom`` with the open disk of radius r about (cx, cy) cut out (points
    on the circle stay in the domain)."""
    inner = dom.contains

    def contains(x, y):
        return inner(x, y) & ((x - cx) ** 2 + (y - cy) ** 2 >= r * r)
    return dataclasses.replace(dom, name=f"{dom.name}-hole({cx},{cy},{r})", contains=contains,
                               area=None if dom.area is None else dom.area - math.pi * r * r,
                               holes=dom.holes + ((cx, cy, r),))


def flower(R: float = 0.69, amp: float = 0.1, petals: int = 5, hole: float = 0.1) -> Domain:
    """The multiply connected domain of section 6.3's last experiment: a
    smooth flower r(theta) = R + amp cos(petals theta) with a circle of
    radius ``hole`` (diameter 0.2 in the paper) cut out about the origin.
    The paper does not define the flower or the circle's position; these
    are this workload's choices."""
    return dataclasses.replace(with_hole(star(R, amp, petals), 0.0, 0.0, hole),
                               name=f"flower(R={R},a={amp},p={petals},hole={hole})")


def boundary_length(dom: Domain, nquad: int = 1 << 16) -> float:
    """Perimeter of a star-shaped boundary by the periodic trapezoid rule."""
    t = 2 * math.pi * np.arange(nquad) / nquad
    r, dr = dom.radius(t), dom.dradius(t)
    return float(np.mean(np.sqrt(r * r + dr * dr)) * 2 * math.pi)


def boundary_points(dom: Domain, count: int) -> np.ndarray:
    """``count`` points theta_j = 2*pi*j/count on the boundary curve, (count, 2)."""
    t = 2 * math.pi * np.arange(count) / count
    r = dom.radius(t)
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)


def boundary_normals(dom: Domain, count: int) -> np.ndarray:
    """Unit outward normals at the points of ``boundary_points``: the
    tangent r'(cos, sin) + r(-sin, cos) of the counter-clockwise curve
    turned clockwise by a right angle."""
    t = 2 * math.pi * np.arange(count) / count
    r, dr = dom.radius(t), dom.dradius(t)
    tx = dr * np.cos(t) - r * np.sin(t)
    ty = dr * np.sin(t) + r * np.cos(t)
    nrm = np.sqrt(tx * tx + ty * ty)
    return np.stack([ty / nrm, -tx / nrm], axis=1)


def hole_points(hole: tuple, count: int):
    """``count`` points on a hole's circle and the domain's outward normals
    there (pointing into the hole), ((count, 2), (count, 2))."""
    cx, cy, r = hole
    t = 2 * math.pi * np.arange(count) / count
    u = np.stack([np.cos(t), np.sin(t)], axis=1)
    return np.array([cx, cy]) + r * u, -u


# --------------------------------------------------------------------------
# Right-hand sides
# --------------------------------------------------------------------------

def trig_sum_1d(seed: int, terms: int = 32, wmax: float = 40.0):
    """Random trigonometric sum  sum_t a_t cos(w_t x + p_t).

    a ~ N(0,1), w ~ U[0, wmax], p ~ U[0, 2pi), drawn from numpy's PCG64 with
    ``seed``.  Returns a callable f(x).
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(terms)
    w = rng.uniform(0.0, wmax, terms)
    p = rng.uniform(0.0, 2 * math.pi, terms)

    def f(x):
        x = np.asarray(x, dtype=np.float64)
        return np.cos(np.multiply.outer(x, w) + p) @ a
    return f


def trig_sum_2d(seed: int, terms: int = 32, wmax: float = 40.0):
    """2D random trigonometric sum with wave vectors rho*(cos alpha, sin alpha)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(terms)
    rho = rng.uniform(0.0, wmax, terms)
    alpha = rng.uniform(0.0, 2 * math.pi, terms)
    p = rng.uniform(0.0, 2 * math.pi, terms)
    wx, wy = rho * np.cos(alpha), rho * np.sin(alpha)

    def f(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        return np.cos(np.multiply.outer(x, wx) + np.multiply.outer(y, wy) + p) @ a
    return f


# --------------------------------------------------------------------------
# Problems
# --------------------------------------------------------------------------

APPROX, POISSON, HELMHOLTZ = 0, 1, 2


@dataclasses.dataclass
class Problem:
    """One least-squares RBF problem on the box [-T, T)^dim.

    n      centres per axis (N = n^dim unknowns); in 2D along x
    s      oversampling factor per axis (L = s*n grid points per axis)
    T      half-width of the periodic box; in 2D along x
    ny, Ty 2D only: centres and half-width along y (None: n and T)
    eh     shape parameter times centre spacing, eps*h (eps = eh / h)
    op     APPROX: rows phi_j(x_i).  POISSON/HELMHOLTZ: interior rows of
           -(Laplacian + k2) phi_j, boundary rows phi_j at boundary points.
    rhs    list of callables f(x) or f(x, y) giving interior data
    bnd    for BVPs, callables g giving Dirichlet data (same length as rhs)
    nb     number of boundary points (BVPs): on the outer curve
           (``boundary_points``), the last ``nb_hole`` of them on the holes
    bc_outer, bc_hole
           boundary condition of the points on the outer curve and on the
           holes: "D" (Dirichlet, rows phi_j) or "N" (Neumann, rows of the
           normal derivative); in 1D one letter per end ("DN": Dirichlet at
           the left end) or one for both
    bnd_n  for Neumann points, callables h(x, y, nx, ny) (1D: h(x, nx)) giving
           the normal derivative data (same length as rhs; None: zero)
    """
    name: str
    dim: int
    n: int
    s: int
    T: float
    eh: float
    domain: Domain
    rhs: list
    op: int = APPROX
    k2: float = 0.0
    bnd: Optional[list] = None
    nb: int = 0
    bweight: float = 1.0
    exact: Optional[list] = None      # exact solutions u (BVPs) for error checks
    k: int = 0                        # sketch width (0: solver's estimate)
    p: int = 10                       # sketch oversampling
    seed: int = 42                    # sketch seed
    ny: Optional[int] = None          # 2D: centres along y (None: n)
    Ty: Optional[float] = None        # 2D: half-width along y (None: T)
    nb_hole: int = 0                  # boundary points on the holes (last nb_hole of nb)
    bc_outer: str = "D"
    bc_hole: str = "D"
    bnd_n: Optional[list] = None

    @property
    def h(self) -> float:
        """Centre spacing along x (the shape parameter is eh / h)."""
        return 2 * self.T / self.n

    @property
    def eps(self) -> float:
        return self.eh / self.h

    @property
    def n_y(self) -> int:
        return self.n if self.ny is None else self.ny

    @property
    def T_y(self) -> float:
        return self.T if self.Ty is None else self.Ty

    def axes(self):
        """[(n, T) per axis]."""
        return [(self.n, self.T)] if self.dim == 1 else [(self.n, self.T), (self.n_y, self.T_y)]

    @property
    def N(self) -> int:
        return self.n if self.dim == 1 else self.n * self.n_y

    def bpoints(self) -> np.ndarray:
        return self._boundary()[0]

    def bnormals(self) -> np.ndarray:
        """Unit outward normals at the boundary points, (nb, dim)."""
        return self._boundary()[1]

    def btypes(self) -> np.ndarray:
        """0 (Dirichlet) or 1 (Neumann) per boundary point, uint8."""
        if self.dim == 1:
            bc = self.bc_outer * 2 if len(self.bc_outer) == 1 else self.bc_outer
            return np.array([c == "N" for c in bc[: self.nb]], dtype=np.uint8)
        nout = self.nb - self.nb_hole
        return np.array([self.bc_outer == "N"] * nout + [self.bc_hole == "N"] * self.nb_hole, dtype=np.uint8)

    @property
    def has_neumann(self) -> bool:
        return bool(self.nb) and bool(np.any(self.btypes()))

    def _boundary(self):
        if self.nb == 0:
            return np.zeros((0, self.dim)), np.zeros((0, self.dim))
        if self.dim == 1:
            return np.array([[-1.0], [1.0]])[: self.nb], np.array([[-1.0], [1.0]])[: self.nb]
        nout = self.nb - self.nb_hole
        pts = [boundary_points(self.domain, nout)]
        nrm = [boundary_normals(self.domain, nout)]
        holes = self.domain.holes
        if self.nb_hole:
            if not holes:
                raise ValueError("nb_hole > 0 on a domain without holes")
            per = [self.nb_hole // len(holes) + (i < self.nb_hole % len(holes)) for i in range(len(holes))]
            for hole, c in zip(holes, per):
                p, q = hole_points(hole, c)
                pts.append(p)
                nrm.append(q)
        return np.concatenate(pts, axis=0), np.concatenate(nrm, axis=0)

    def bdata(self, i: int, bp: Optional[np.ndarray] = None) -> np.ndarray:
        """Boundary data of right-hand side i at the boundary points:
        g (Dirichlet points) or the normal derivative h (Neumann points)."""
        bp = self.bpoints() if bp is None else bp
        types = self.btypes()
        out = np.zeros(bp.shape[0])
        d = types == 0
        if np.any(d):
            out[d] = self.bnd[i](*bp[d].T)
        if np.any(~d) and self.bnd_n is not None:
            nv = self.bnormals()
            out[~d] = self.bnd_n[i](*bp[~d].T, *nv[~d].T)
        return out


def _f_c1(x):
    return np.exp(x) * np.sin(7 * x) + x * x


def config_c1(n: int = 256) -> Problem:
    """1D plain AZ, eps = 1/h, Omega = [-0.5, 0.5], f = e^x sin 7x + x^2."""
    return Problem("C1", 1, n, 2, 1.0, 1.0, interval(-0.5, 0.5), [_f_c1], k=32)


def config_c1a(n: int = 256) -> Problem:
    """C1 at eps*h = 0.5, the regime where FP64 AZ reaches residual 1e-10."""
    return Problem("C1a", 1, n, 2, 1.0, 0.5, interval(-0.5, 0.5), [_f_c1], k=32)


def family_1d(n: int, nrhs: int, eh: float = 0.5, seed0: int = 1000,
              name: str = "C2") -> Problem:
    """1D batched family: random trig sums on [-0.5, 0.5], box [-1, 1)."""
    return Problem(name, 1, n, 2, 1.0, eh, interval(-0.5, 0.5),
                   [trig_sum_1d(seed0 + i) for i in range(nrhs)], k=32)


def config_c2(n: int = 65536, nrhs: int = 64) -> Problem:
    return family_1d(n, nrhs)


def _f_c3(x, y):
    return np.cos(3 * x + 2 * y) * np.exp(-x * x)


def config_c3(n: int = 128, eh: float = 1.0) -> Problem:
    """2D approximation on the disk of radius 0.8, f = cos(3x+2y) exp(-x^2)."""
    return Problem("C3" if eh == 1.0 else "C3a", 2, n, 2, 1.0, eh, disk(0.8),
                   [_f_c3], p=10)


def config_c3a(n: int = 128) -> Problem:
    return config_c3(n, 0.5)


def _f_e6(nx, ny):
    def f(x, y):
        return np.sin(nx / 10.0 * x + ny / 10.0 * y)
    return f


def config_ellipse(nx: int = 128, ny: int = 64, eh: Optional[float] = None) -> Problem:
    """Section 5.4's non-periodic experiment on an anisotropic box: the
    ellipse x^2 + 4 y^2 <= 1 in [-1.4, 1.4] x [-0.7, 0.7] (equal spacing on
    both axes when ny = nx / 2), s = 2, f = sin(nx x / 10 + ny y / 10), shape
    parameter from tau0 = 1e-5 unless eh is given."""
    return Problem(f"ellipse{nx}x{ny}", 2, nx, 2, 1.4, shape_parameter_eh(1e-5) if eh is None else eh,
                   ellipse(1.0, 0.5), [_f_e6(nx, ny)], ny=ny, Ty=0.7, p=10)


def _u_c4(x, y):
    return np.sin(2 * x) * np.cos(3 * y)


def _f_c4(x, y):
    return 13.0 * np.sin(2 * x) * np.cos(3 * y)


def config_c4(n: int = 256, eh: float = 0.5, R: float = 0.7) -> Problem:
    """2D Poisson -Lap u = f on the star 0.7 + 0.1 cos 5 theta, weak Dirichlet.

    Boundary points: round(4 * length / h), equispaced in theta.
    """
    dom = star(R)
    h = 2.0 / n
    nb = int(round(4 * boundary_length(dom) / h))
    return Problem("C4", 2, n, 2, 1.0, eh, dom, [_f_c4], op=POISSON, k2=0.0,
                   bnd=[_u_c4], nb=nb, exact=[_u_c4], p=10)


def _f_flower(x, y):
    # -(Lap + 4) u = -exp(-4((x+0.3)^2 + y^2)^2): the source of section 6.3's
    # last experiment written for the operator -(Lap + k2)
    return -np.exp(-4.0 * ((x + 0.3) ** 2 + y * y) ** 2)


def _u_flower_m(x, y):
    return np.sin(2 * x) * np.cos(3 * y) + 0.5 * x * y


def _f_flower_m(x, y):
    # -(Lap + 4) u with Lap(sin 2x cos 3y) = -13 sin 2x cos 3y, Lap(x y) = 0
    return 9.0 * np.sin(2 * x) * np.cos(3 * y) - 2.0 * x * y


def _dn_flower_m(x, y, nx, ny):
    ux = 2 * np.cos(2 * x) * np.cos(3 * y) + 0.5 * y
    uy = -3 * np.sin(2 * x) * np.sin(3 * y) + 0.5 * x
    return ux * nx + uy * ny


def config_flower(n: int = 128, eh: float = 0.5, manufactured: bool = False,
                  nb_outer: int = 200, nb_hole: int = 100) -> Problem:
    """Section 6.3's last experiment: Helmholtz (Lap + 4) u = exp(-4((x+0.3)^2
    + y^2)^2) on the flower with a hole (``flower``), homogeneous Neumann
    data on the outer curve and homogeneous Dirichlet data on the circle,
    200 and 100 boundary points, box [-1, 1]^2, s = 2.  The paper uses
    100 x 100 centres; n is a power of two here.  ``manufactured`` swaps in
    u = sin 2x cos 3y + xy/2 with its source, normal derivative (outer curve)
    and values (circle), for error checks."""
    dom = flower()
    common = dict(op=HELMHOLTZ, k2=4.0, nb=nb_outer + nb_hole, nb_hole=nb_hole,
                  bc_outer="N", bc_hole="D", p=10)
    if manufactured:
        return Problem("E9m", 2, n, 2, 1.0, eh, dom, [_f_flower_m], bnd=[_u_flower_m],
                       bnd_n=[_dn_flower_m], exact=[_u_flower_m], **common)
    return Problem("E9", 2, n, 2, 1.0, eh, dom, [_f_flower], bnd=[lambda x, y: 0.0 * x],
                   bnd_n=[lambda x, y, nx, ny: 0.0 * x], **common)


# --------------------------------------------------------------------------
# Test points
# --------------------------------------------------------------------------

def test_points(prob: Problem, m1d: int = 4096, m2d: int = 1024) -> np.ndarray:
    """Fine test set: 1D linspace over the interval, 2D a cell-centred
    m2d x m2d lattice on the box [-T, T] x [-T_y, T_y] intersected with the
    domain."""
    if prob.dim == 1:
        lo, hi = prob.domain.bounds
        if prob.domain.name == "box":
            return np.linspace(lo, hi, m1d, endpoint=False)[:, None]
        return np.linspace(lo, hi, m1d)[:, None]
    t = -prob.T + (np.arange(m2d) + 0.5) * (2.0 * prob.T / m2d)
    u = -prob.T_y + (np.arange(m2d) + 0.5) * (2.0 * prob.T_y / m2d)
    X, Y = np.meshgrid(t, u, indexing="ij")
    keep = prob.domain.contains(X, Y)
    return np.stack([X[keep], Y[keep]], axis=1)


# --------------------------------------------------------------------------
# Served request stream
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds from stream start
    problem: Problem


def served_stream(count: int = 512, seed: int = 2024, rate: float = 100.0,
                  frac_1d: float = 0.7, max_rhs: int = 16, eh: float = 0.5,
                  sides=(64, 128, 256), exps=range(10, 17)) -> list:
    """Poisson-arrival stream of mixed 1D / 2D approximation requests.

    1D: N = 2^e with e uniform in ``exps``.  2D: side uniform in ``sides``,
    disk or star with radius uniform in [0.6, 0.85].  Each request carries
    1..max_rhs random trigonometric right-hand sides.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    exps = list(exps)
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        nrhs = int(rng.integers(1, max_rhs + 1))
        rseed = int(rng.integers(0, 2**31 - 1))
        if rng.uniform() < frac_1d:
            n = 2 ** int(rng.choice(exps))
            prob = Problem(f"req{rid}-1d", 1, n, 2, 1.0, eh, interval(-0.5, 0.5),
                           [trig_sum_1d(rseed + i) for i in range(nrhs)], k=32,
                           seed=rseed)
        else:
            n = int(rng.choice(list(sides)))
            R = float(rng.uniform(0.6, 0.85))
            dom = disk(R) if rng.uniform() < 0.5 else star(R)
            prob = Problem(f"req{rid}-2d", 2, n, 2, 1.0, eh, dom,
                           [trig_sum_2d(rseed + i) for i in range(nrhs)],
                           seed=rseed)
        out.append(Request(rid, t, prob))
    return out
