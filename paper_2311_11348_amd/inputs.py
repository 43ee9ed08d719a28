"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds no arithmetic of the discontinuous Galerkin method: it builds
triangulations, vertex bathymetry, point-wise initial conditions, boundary
forcing parameters and random modal coefficient arrays.  Everything the method
computes from these inputs lives either in the HIP library or in the oracle.

Workloads (all distances in metres, times in seconds):

* ``c1``  32x32x2 structured mesh of a 100 km square, flat 10 m depth, 0.1 m
          Gaussian bump of width 10 km at the centre, land walls, p = 1.
* ``c2``  512x512x2 mesh jittered by U(-0.2h, 0.2h) (seed 2), smooth
          sin*cos bathymetry between 10 and 4000 m, lake at rest, west edge
          open and forced by a 0.5 m tide of period 44712 s, p = 2.
* ``c3``  256x256x2 jittered mesh (seed 3), linear shelf 4000 m -> 50 m,
          2 m hump of width 20 km at (L/4, L/2), land walls, p in {1,2,3}.
* ``c4``  64 independent instances (seed 4, instance i seed 4000+i).
* ``c5``  Poisson request trace at 20 req/s for 120 s (seed 5).

The Bahamas bathymetry and mesh used in the paper's tidal test (Sec. "Tidal
flow at Bahamas with water hump") are not available; ``c2``/``c3`` stand in
with synthetic shapes of the same kind (tidal forcing, deep-to-shallow shelf).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

L_DOMAIN = 1.0e5
G_EARTH = 9.81
TIDE_PERIOD = 44712.0
# Physical constants of the tidal setup (Tab. physical_quantities).
CORIOLIS_BAHAMAS = 3.19e-5
CF_BAHAMAS = 0.009

FRICTION_NONE = 0
FRICTION_LINEAR = 1
FRICTION_QUADRATIC = 2

TAG_INTERIOR = -1
TAG_LAND = 0
TAG_OPEN = 1

K_OF_P = (1, 3, 6, 10)


@dataclass
class Mesh:
    """Triangulation with counter-clockwise triangles.

    ``tag[e, k]`` is the boundary tag of the local edge k of element e, the
    edge opposite vertex k (joining vertices k+1 and k+2 mod 3): -1 for an
    edge that should have a neighbour, 0 for land, 1 for open sea.
    """
    vxy: np.ndarray          # [nv, 2] float64
    tri: np.ndarray          # [ne, 3] int32
    tag: np.ndarray          # [ne, 3] int8
    n: int = 0
    length: float = L_DOMAIN

    @property
    def nv(self) -> int:
        return int(self.vxy.shape[0])

    @property
    def ne(self) -> int:
        return int(self.tri.shape[0])

    def areas(self) -> np.ndarray:
        p = self.vxy[self.tri]
        d1 = p[:, 1] - p[:, 0]
        d2 = p[:, 2] - p[:, 0]
        return 0.5 * (d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])

    def centroids(self) -> np.ndarray:
        return self.vxy[self.tri].mean(axis=1)

    def inscribed_diameters(self) -> np.ndarray:
        p = self.vxy[self.tri]
        per = (np.linalg.norm(p[:, 1] - p[:, 0], axis=1)
               + np.linalg.norm(p[:, 2] - p[:, 1], axis=1)
               + np.linalg.norm(p[:, 0] - p[:, 2], axis=1))
        return 4.0 * self.areas() / per


def structured_mesh(n: int, length: float = L_DOMAIN, jitter: float = 0.0,
                    seed: Optional[int] = None, open_west: bool = False) -> Mesh:
    """n x n squares, each cut along its SW->NE diagonal into two triangles.

    Vertices are numbered row-major (x fastest); squares likewise, two
    elements per square.  With ``jitter`` > 0 every vertex draws an offset
    U(-jitter*h, jitter*h) in x and y from ``default_rng(seed)`` in row-major
    order and only interior vertices apply it, so boundary vertices stay put.
    Local edge k is opposite vertex k.  Boundary edges on x = 0 get tag 1
    (open) if ``open_west`` else 0; all other boundary edges are land.
    """
    h = length / n
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    vxy = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        off = rng.uniform(-jitter * h, jitter * h, size=((n + 1) * (n + 1), 2))
        interior = ((ii.ravel() > 0) & (ii.ravel() < n) & (jj.ravel() > 0) & (jj.ravel() < n))
        vxy[interior] += off[interior]
    jj2, ii2 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")   # square (i, j), i fastest
    i1, j1 = ii2.ravel(), jj2.ravel()
    a = j1 * (n + 1) + i1           # SW
    b = a + 1                       # SE
    c = a + n + 2                   # NE
    d = a + n + 1                   # NW
    tri = np.empty((2 * n * n, 3), dtype=np.int32)
    tri[0::2] = np.stack([a, b, c], 1)   # lower-right (SW, SE, NE): edge 2 south, edge 0 east
    tri[1::2] = np.stack([a, c, d], 1)   # upper-left (SW, NE, NW): edge 0 north, edge 1 west
    tag = np.full((2 * n * n, 3), TAG_INTERIOR, dtype=np.int8)
    lo, up = tag[0::2], tag[1::2]
    lo[j1 == 0, 2] = TAG_LAND
    lo[i1 == n - 1, 0] = TAG_LAND
    up[j1 == n - 1, 0] = TAG_LAND
    up[i1 == 0, 1] = TAG_OPEN if open_west else TAG_LAND
    tag[0::2], tag[1::2] = lo, up
    m = Mesh(vxy=vxy, tri=tri, tag=tag, n=n, length=length)
    if not np.all(m.areas() > 0.0):
        raise ValueError("jitter produced a non-positive triangle area")
    return m


# ---------------------------------------------------------------- bathymetry
def bathy_flat(depth: float) -> Callable[[np.ndarray, np.ndarray], np.ndarray]:
    return lambda x, y: np.full_like(np.asarray(x, dtype=np.float64), depth)


def bathy_sincos(length: float = L_DOMAIN) -> Callable:
    """10 m + 3990 m * (1 + sin(2 pi x/L) cos(2 pi y/L)) / 2."""
    return lambda x, y: 10.0 + 3990.0 * (1.0 + np.sin(2 * np.pi * x / length)
                                         * np.cos(2 * np.pi * y / length)) / 2.0


def bathy_shelf(length: float = L_DOMAIN, deep: float = 4000.0, shallow: float = 50.0) -> Callable:
    """Linear in x from ``deep`` at x = 0 to ``shallow`` at x = L."""
    return lambda x, y: deep + (shallow - deep) * np.asarray(x) / length


def bathy_random_smooth(rng: np.random.Generator, length: float = L_DOMAIN,
                        lo: float = 50.0, hi: float = 4000.0, nterms: int = 4) -> Callable:
    """lo + (hi-lo) * minmax(sum_k a_k sin(2 pi (m_k x + n_k y)/L + phi_k)).

    The min-max scaling uses the extremes of the sum sampled on a 257x257 grid,
    then clips, so every vertex depth lies in [lo, hi].
    """
    a = rng.uniform(0.5, 1.0, nterms)
    mn = []
    while len(mn) < nterms:
        m_, n_ = rng.integers(0, 4, 2)
        if m_ == 0 and n_ == 0:
            continue
        mn.append((int(m_), int(n_)))
    phi = rng.uniform(0.0, 2 * np.pi, nterms)

    def raw(x, y):
        s = np.zeros_like(np.asarray(x, dtype=np.float64))
        for k in range(nterms):
            s = s + a[k] * np.sin(2 * np.pi * (mn[k][0] * x + mn[k][1] * y) / length + phi[k])
        return s
    g = np.linspace(0.0, length, 257)
    gx, gy = np.meshgrid(g, g)
    r = raw(gx, gy)
    rmin, rmax = float(r.min()), float(r.max())

    def f(x, y):
        t = (raw(x, y) - rmin) / (rmax - rmin)
        return lo + (hi - lo) * np.clip(t, 0.0, 1.0)
    return f


# --------------------------------------------------------- initial conditions
def ic_gaussian(amp: float, width: float, x0: float, y0: float) -> Callable:
    """xi = amp * exp(-r^2 / width^2), U = V = 0."""
    def f(x, y):
        r2 = (np.asarray(x) - x0) ** 2 + (np.asarray(y) - y0) ** 2
        xi = amp * np.exp(-r2 / (width * width))
        z = np.zeros_like(xi)
        return xi, z, z.copy()
    return f


def ic_rest(level: float = 0.0) -> Callable:
    def f(x, y):
        xi = np.full_like(np.asarray(x, dtype=np.float64), level)
        z = np.zeros_like(xi)
        return xi, z, z.copy()
    return f


def ic_dambreak() -> Callable:
    """Radial dam break of Sec. "Radial dam break" on [0,5]^2."""
    def f(x, y):
        r2 = (np.asarray(x) - 2.5) ** 2 + (np.asarray(y) - 2.5) ** 2
        xi = np.where(r2 < 0.25, 2.0 + 0.5 * np.exp(-15.0 * r2), 1.0)
        z = np.zeros_like(xi)
        return xi, z, z.copy()
    return f


# ------------------------------------------------------------------- configs
@dataclass
class Forcing:
    """Open-sea elevation xi_hat(t) = sum_i amp_i sin(omega_i t + phase_i)."""
    amp: list = field(default_factory=list)
    omega: list = field(default_factory=list)
    phase: list = field(default_factory=list)

    def __call__(self, t: float) -> float:
        return float(sum(a * math.sin(w * t + p) for a, w, p in zip(self.amp, self.omega, self.phase)))


def tide_forcing(amp: float = 0.5, period: float = TIDE_PERIOD) -> Forcing:
    return Forcing([amp], [2 * math.pi / period], [0.0])


@dataclass
class Problem:
    name: str
    mesh: Mesh
    hb_vertex: np.ndarray
    ic: Callable
    p: np.ndarray                 # per-element order (int8)
    p_base: int
    p_max: int
    g: float = G_EARTH
    f_coriolis: float = 0.0
    friction: int = FRICTION_NONE
    friction_coef: float = 0.0
    forcing: Forcing = field(default_factory=Forcing)
    steps: int = 100
    cfl: float = 0.2
    adapt: int = 0
    adapt_tau: float = 1e-3
    bathy: Optional[Callable] = None
    dt_fixed: Optional[float] = None   # a prescribed step instead of the CFL rule
    h_min: float = 0.0                 # minimum depth control after every stage (0: off)

    def dt(self) -> float:
        """Fixed step from the analytic initial state at the vertices and centroids.

        dt = CFL * min_e d_e / ((2 p_max + 1) * max(|u0| + sqrt(g H0))), with d_e
        the inscribed-circle diameter.  Only point values of the initial
        condition and bathymetry are used.  ``dt_fixed``, when set, is returned
        instead.
        """
        if self.dt_fixed is not None:
            return float(self.dt_fixed)
        pts = np.concatenate([self.mesh.vxy, self.mesh.centroids()], axis=0)
        xi, U, V = self.ic(pts[:, 0], pts[:, 1])
        if self.bathy is not None:
            hb = self.bathy(pts[:, 0], pts[:, 1])
        else:
            hb = np.full(pts.shape[0], float(self.hb_vertex.mean()))
        H = xi + hb
        speed = np.sqrt(U * U + V * V) / H + np.sqrt(self.g * H)
        return float(self.cfl * self.mesh.inscribed_diameters().min()
                     / ((2 * self.p_max + 1) * speed.max()))


def _problem(name, mesh, bathy, ic, p, p_base, p_max, **kw) -> Problem:
    hb = bathy(mesh.vxy[:, 0], mesh.vxy[:, 1]).astype(np.float64)
    pe = np.full(mesh.ne, p, dtype=np.int8) if np.isscalar(p) else np.asarray(p, np.int8)
    return Problem(name=name, mesh=mesh, hb_vertex=hb, ic=ic, p=pe, p_base=p_base,
                   p_max=p_max, bathy=bathy, **kw)


def config_c1(n: int = 32, p: int = 1) -> Problem:
    mesh = structured_mesh(n)
    return _problem("c1", mesh, bathy_flat(10.0), ic_gaussian(0.1, 1.0e4, L_DOMAIN / 2, L_DOMAIN / 2),
                    p, p, p, steps=100)


def config_shallow(n: int = 24, p: int = 2, h_min: float = 0.25, seed: int = 8) -> Problem:
    """Shallow water for the minimum depth control: bottom 1 m deep at x = 0
    and 0.5 m at x = L, at rest with a Gaussian depression of the surface
    (-0.6 m, width 15 km) in the middle, 0.15 m deep at its centre; all land,
    jittered mesh."""
    mesh = structured_mesh(n, jitter=0.2, seed=seed)
    return _problem("shallow", mesh, bathy_shelf(deep=1.0, shallow=0.5),
                    ic_gaussian(-0.6, 1.5e4, L_DOMAIN / 2, L_DOMAIN / 2), p, min(p, 1), p, steps=20,
                    h_min=h_min)


def config_c2(n: int = 512, p: int = 2, seed: int = 2) -> Problem:
    mesh = structured_mesh(n, jitter=0.2, seed=seed, open_west=True)
    return _problem("c2", mesh, bathy_sincos(), ic_rest(0.0), p, min(p, 1), p,
                    f_coriolis=CORIOLIS_BAHAMAS, friction=FRICTION_QUADRATIC,
                    friction_coef=CF_BAHAMAS, forcing=tide_forcing(), steps=500)


def config_c3(n: int = 256, seed: int = 3) -> Problem:
    mesh = structured_mesh(n, jitter=0.2, seed=seed)
    return _problem("c3", mesh, bathy_shelf(), ic_gaussian(2.0, 2.0e4, L_DOMAIN / 4, L_DOMAIN / 2),
                    1, 1, 3, f_coriolis=CORIOLIS_BAHAMAS, friction=FRICTION_QUADRATIC,
                    friction_coef=CF_BAHAMAS, steps=1000, adapt=1, adapt_tau=1e-3)


DAMBREAK_LENGTH = 5.0
DAMBREAK_DT = 1.0e-5


def config_dambreak(n: int = 1024, p_lo: int = 1, p_hi: int = 2, every: int = 32, seed: int = 6,
                    dt_fixed: Optional[float] = DAMBREAK_DT, adapt_tau: Optional[float] = None) -> Problem:
    """Radial dam break of Sec. "Radial dam break" with the physical values of
    its table of physical quantities: [0,5]^2, g = 1, constant bathymetry
    0.5 m, walls on every side, Coriolis 1e-5 1/s, linear friction
    tau_bf = 1e-4 H (that is -1e-4 q), the discontinuous radial elevation at
    rest.  The mesh is the n x n x 2 triangulation with interior nodes
    jittered by U(-0.2h, 0.2h) (n = 1024: 2,097,152 triangles, the count
    the paper measures on).  Orders: p_lo everywhere and p_hi on every
    ``every``-th element in mesh order (the statically adaptive setups;
    every = 1 gives uniform p_hi, every = 0 uniform p_lo), base order p_lo.
    Time step: the static runs' 1e-5 s unless ``dt_fixed`` is None (then the
    CFL rule).  With ``adapt_tau`` the orders are dynamic instead (the
    dynamic runs): every element starts at p_lo and the order update before
    each step sets p_lo..p_hi from the indicator with threshold adapt_tau."""
    mesh = structured_mesh(n, length=DAMBREAK_LENGTH, jitter=0.2, seed=seed)
    p = np.full(mesh.ne, p_lo, np.int8)
    if adapt_tau is None and every > 0:
        p[::every] = p_hi
    p_max = int(p.max()) if adapt_tau is None else p_hi
    return _problem(f"dambreak{n}", mesh, bathy_flat(0.5), ic_dambreak(), p, min(p_lo, p_max), p_max, g=1.0,
                    f_coriolis=1.0e-5, friction=FRICTION_LINEAR, friction_coef=1.0e-4, steps=100,
                    dt_fixed=dt_fixed, adapt=0 if adapt_tau is None else 1,
                    adapt_tau=1e-3 if adapt_tau is None else adapt_tau)


def instance_mesh_n(n_elements: float) -> int:
    """Side count n of the n x n x 2 mesh closest to ``n_elements`` triangles."""
    return max(2, int(round(math.sqrt(n_elements / 2.0))))


def instance_problem(rng: np.random.Generator, n_elements: float, p: int, tidal: bool, steps: int,
                     name: str) -> Problem:
    """A batched/served instance: ~n_elements jittered triangles of the 100 km
    square, uniform order p, smooth random bathymetry 50-4000 m, Coriolis and
    quadratic friction; tidal (lake at rest, west edge open, 0.5 m tide) or a
    2 m Gaussian hump in a closed basin.  The mesh seed and the bathymetry are
    drawn from ``rng``."""
    n = instance_mesh_n(n_elements)
    mesh = structured_mesh(n, jitter=0.2, seed=int(rng.integers(0, 2**31 - 1)), open_west=tidal)
    bathy = bathy_random_smooth(rng)
    if tidal:
        ic, forcing = ic_rest(0.0), tide_forcing()
    else:
        ic, forcing = ic_gaussian(2.0, 2.0e4, L_DOMAIN / 4, L_DOMAIN / 2), Forcing()
    return _problem(name, mesh, bathy, ic, p, p, p, f_coriolis=CORIOLIS_BAHAMAS,
                    friction=FRICTION_QUADRATIC, friction_coef=CF_BAHAMAS, forcing=forcing,
                    steps=steps)


def config_instance(seed: int, n_lo: float = 16e3, n_hi: float = 500e3) -> Problem:
    """One batched instance: log-uniform size, p in {1,2,3}, tidal or hump, 300 steps."""
    rng = np.random.default_rng(seed)
    N = math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))
    p = int(rng.integers(1, 4))
    tidal = bool(rng.integers(0, 2) == 0)
    return instance_problem(rng, N, p, tidal, 300, f"inst{seed}")


def config_c4(count: int = 64, seed: int = 4) -> list:
    return [config_instance(seed * 1000 + i) for i in range(count)]


@dataclass
class Request:
    arrival: float
    seed: int
    n_elements_target: float
    p: int
    steps: int
    tidal: bool


def request_trace(rate: float = 20.0, duration: float = 120.0, seed: int = 5,
                  n_lo: float = 8e3, n_hi: float = 260e3) -> list:
    """Poisson arrivals; request i draws its own parameters from seed 5000+i."""
    rng = np.random.default_rng(seed)
    t, out, i = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        r = np.random.default_rng(seed * 1000 + i)
        N = math.exp(r.uniform(math.log(n_lo), math.log(n_hi)))
        out.append(Request(arrival=t, seed=seed * 1000 + i, n_elements_target=N,
                           p=int(r.integers(1, 4)), steps=int(r.integers(200, 2001)),
                           tidal=bool(r.integers(0, 2) == 0)))
        i += 1
    return out


def request_problem(req: Request) -> Problem:
    """The solve a served request describes: ~n_elements jittered triangles
    (mesh seed from the request's seed), uniform order p; tidal requests take
    the tidal workload's bathymetry, forcing and open west edge, hump requests
    the tsunami workload's shelf and 2 m hump in a closed basin."""
    rng = np.random.default_rng([req.seed, 1])
    mesh = structured_mesh(instance_mesh_n(req.n_elements_target), jitter=0.2,
                           seed=int(rng.integers(0, 2**31 - 1)), open_west=req.tidal)
    if req.tidal:
        bathy, ic, forcing = bathy_sincos(), ic_rest(0.0), tide_forcing()
    else:
        bathy, ic, forcing = bathy_shelf(), ic_gaussian(2.0, 2.0e4, L_DOMAIN / 4, L_DOMAIN / 2), Forcing()
    return _problem(f"req{req.seed}", mesh, bathy, ic, req.p, req.p, req.p, f_coriolis=CORIOLIS_BAHAMAS,
                    friction=FRICTION_QUADRATIC, friction_coef=CF_BAHAMAS, forcing=forcing,
                    steps=req.steps)


# ------------------------------------------------------------- random states
def random_state(mesh: Mesh, p: np.ndarray, p_max: int, seed: int, hb_vertex: np.ndarray,
                 xi_amp: float = 0.5, q_amp: float = 1.0, decay: float = 0.3) -> np.ndarray:
    """Random modal coefficients [ne][3][K(p_max)] in the physical orthonormal basis.

    The element mean of each field is drawn uniformly in [-amp, amp] and
    stored as mean * sqrt(area) (the first orthonormal basis function is
    1/sqrt(area)); higher modes get amp * decay^degree * sqrt(area) * N(0,1).
    Modes above K(p_e) are zero.  ``xi_amp`` must stay well below the minimum
    depth so that the total depth is positive everywhere.
    """
    rng = np.random.default_rng(seed)
    K = K_OF_P[p_max]
    ne = mesh.ne
    sa = np.sqrt(mesh.areas())
    deg = np.array([0, 1, 1, 2, 2, 2, 3, 3, 3, 3][:K])
    amps = np.array([xi_amp, q_amp, q_amp])
    c = np.zeros((ne, 3, K))
    c[:, :, 0] = rng.uniform(-1.0, 1.0, (ne, 3)) * amps[None, :] * sa[:, None]
    hi = rng.standard_normal((ne, 3, K)) * (amps[None, :, None] * decay ** deg[None, None, :]) * sa[:, None, None]
    c[:, :, 1:] = hi[:, :, 1:]
    kk = np.asarray([K_OF_P[int(x)] for x in p])
    mask = np.arange(K)[None, :] < kk[:, None]
    c *= mask[:, None, :]
    return c
