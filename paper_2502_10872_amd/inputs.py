"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module produces geometry only: rest positions, triangle lists, pinned-vertex
masks, random rigid motions and perturbations.  It contains none of the bending
model's arithmetic (no operators, areas, masses or forces); both the CPU oracle
and the HIP library derive those themselves from what is generated here.

Meshes follow the paper's setting of a triangulated mid-surface with positions
x = X + u (Sec. 4.1, eq. 3).  Workload recipes:

* plate: flat n x n grid on [0, Lx] x [0, Ly], each quad split along (i,j)->(i+1,j+1),
  counter-clockwise in the parameter plane;
* cylinder patch: the grid wrapped onto a cylinder of radius R about the y-axis,
  rest position (R sin(u/R), v, R cos(u/R) - R) with u centred on 0;
* sphere cap: the grid on a square of side S, lifted vertically onto a sphere of
  radius R, z = sqrt(R^2 - r^2) - R;
* equilateral: rows of equilateral triangles (odd rows shifted by half a spacing);
* jitter: interior vertices only, uniform in-plane offsets in (-a*l, a*l)^2 drawn
  with NumPy's PCG64 from a stated seed, applied before the map to 3D.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MODELS = ("EP", "ES", "FP", "FS", "SP", "SS")
MODEL_ID = {m: i for i, m in enumerate(MODELS)}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def grid_tris(nx: int, ny: int) -> np.ndarray:
    """Triangles of an nx-by-ny vertex grid (vertex id = j*nx + i), diagonal (i,j)->(i+1,j+1)."""
    if nx < 2 or ny < 2:
        return np.zeros((0, 3), dtype=np.int32)
    i, j = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    v00 = j * nx + i
    v10 = v00 + 1
    v01 = v00 + nx
    v11 = v01 + 1
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    tris = np.empty((2 * len(v00), 3), dtype=np.int32)
    tris[0::2] = t1
    tris[1::2] = t2
    return tris


def grid_uv(nx: int, ny: int, lx: float, ly: float) -> np.ndarray:
    u = np.linspace(0.0, lx, nx)
    v = np.linspace(0.0, ly, ny)
    uu, vv = np.meshgrid(u, v, indexing="xy")
    return np.stack([uu.ravel(), vv.ravel()], axis=1)


def grid_boundary_mask(nx: int, ny: int) -> np.ndarray:
    i = np.tile(np.arange(nx), ny)
    j = np.repeat(np.arange(ny), nx)
    return (i == 0) | (i == nx - 1) | (j == 0) | (j == ny - 1)


def jitter_uv(uv: np.ndarray, nx: int, ny: int, spacing: float, amp: float, seed: int) -> np.ndarray:
    """Uniform in-plane jitter of interior grid vertices, |offset| < amp*spacing per axis."""
    if amp == 0.0:
        return uv.copy()
    g = rng(seed)
    off = g.uniform(-amp * spacing, amp * spacing, size=uv.shape)
    off[grid_boundary_mask(nx, ny)] = 0.0
    return uv + off


def flat_from_uv(uv: np.ndarray) -> np.ndarray:
    return np.stack([uv[:, 0], uv[:, 1], np.zeros(len(uv))], axis=1)


def cylinder_from_uv(uv: np.ndarray, radius: float, u_centre: float) -> np.ndarray:
    phi = (uv[:, 0] - u_centre) / radius
    return np.stack([radius * np.sin(phi), uv[:, 1], radius * np.cos(phi) - radius], axis=1)


def sphere_cap_from_uv(uv: np.ndarray, radius: float, centre: tuple[float, float]) -> np.ndarray:
    x = uv[:, 0] - centre[0]
    y = uv[:, 1] - centre[1]
    r2 = x * x + y * y
    if np.any(r2 >= radius * radius):
        raise ValueError("sphere cap square does not fit inside the sphere")
    return np.stack([x, y, np.sqrt(radius * radius - r2) - radius], axis=1)


def equilateral_mesh(nx: int, ny: int, spacing: float = 1.0):
    """Vertex rows of equilateral triangles; returns (X [nv,3], tris [nt,3]) counter-clockwise."""
    xs = []
    for j in range(ny):
        shift = 0.5 * spacing if (j % 2) else 0.0
        for i in range(nx):
            xs.append((i * spacing + shift, j * spacing * math.sqrt(3.0) / 2.0, 0.0))
    X = np.array(xs, dtype=np.float64)
    tris = []
    for j in range(ny - 1):
        for i in range(nx - 1):
            a = j * nx + i
            b = a + 1
            c = a + nx
            d = c + 1
            if j % 2 == 0:
                tris.append((a, b, c))
                tris.append((b, d, c))
            else:
                tris.append((a, b, d))
                tris.append((a, d, c))
    return X, np.array(tris, dtype=np.int32)


def boundary_edges(tris: np.ndarray) -> np.ndarray:
    """Undirected edges used by exactly one triangle, [n][2] with the smaller vertex id first, sorted."""
    t = np.asarray(tris, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e.sort(axis=1)
    base = int(t.max()) + 1 if len(t) else 1
    u, cnt = np.unique(e[:, 0] * base + e[:, 1], return_counts=True)
    u = u[cnt == 1]
    return np.stack([u // base, u % base], axis=1).astype(np.int32)


def random_rotation(g: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(g.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@dataclass
class Mesh:
    """A synthetic workload: rest positions, triangles, pinned vertices and its recipe."""

    name: str
    X: np.ndarray  # float64 [nv, 3]
    tris: np.ndarray  # int32 [nt, 3]
    pinned: np.ndarray  # uint8 [nv]
    model: str = "EP"
    spacing: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return int(self.X.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tris.shape[0])


def _pins_columns(nx, ny, cols):
    i = np.tile(np.arange(nx), ny)
    return np.isin(i, cols).astype(np.uint8)


def _pins_rows(nx, ny, rows):
    j = np.repeat(np.arange(ny), nx)
    return np.isin(j, rows).astype(np.uint8)


def plate_mesh(n: int, side: float = 1.0, jitter: float = 0.0, seed: int = 0, model: str = "EP",
               pins: str = "clamp_x0") -> Mesh:
    """Flat square plate, n x n vertices.  pins: 'clamp_x0' pins the two vertex columns at x in {0, l}
    (a clamped side held by two rows of fixed nodes), 'ring' pins the boundary, 'none' pins nothing."""
    l = side / (n - 1)
    uv = jitter_uv(grid_uv(n, n, side, side), n, n, l, jitter, seed)
    X = flat_from_uv(uv)
    if pins == "clamp_x0":
        pinned = _pins_columns(n, n, [0, 1])
    elif pins == "ring":
        pinned = grid_boundary_mask(n, n).astype(np.uint8)
    else:
        pinned = np.zeros(n * n, dtype=np.uint8)
    return Mesh(f"plate{n}", X, grid_tris(n, n), pinned, model, l, dict(n=n, side=side, jitter=jitter, seed=seed))


def equilateral_plate(n: int, side: float = 1.0, model: str = "EP") -> Mesh:
    """Flat plate of equilateral triangles with straight sides: rows s sqrt(3)/2 apart, even rows n vertices
    at i s (s = side / (n - 1)), odd rows shifted by s/2 and closed by a vertex on each side, so every side
    triangle is a half triangle; as many rows as make the height nearest the side.  Boundary held (the
    simply supported setting); meta['height'] is the plate's height."""
    s = side / (n - 1)
    hgt = s * math.sqrt(3.0) / 2.0
    ny = int(round(side / hgt)) + 1
    rows, pts = [], []
    for j in range(ny):
        if j % 2 == 0:
            xs = [i * s for i in range(n)]
        else:
            xs = [0.0] + [(k - 0.5) * s for k in range(1, n)] + [(n - 1) * s]
        rows.append(list(range(len(pts), len(pts) + len(xs))))
        pts += [(x, j * hgt, 0.0) for x in xs]
    tris = []
    for j in range(ny - 1):
        lo, hi = rows[j], rows[j + 1]
        if j % 2 == 0:  # even row below, odd row above
            E, Od = lo, hi
            tris.append((E[0], Od[1], Od[0]))
            tris += [(E[i], E[i + 1], Od[i + 1]) for i in range(n - 1)]
            tris += [(E[i + 1], Od[i + 2], Od[i + 1]) for i in range(n - 2)]
            tris.append((E[n - 1], Od[n], Od[n - 1]))
        else:  # odd row below, even row above
            Od, E = lo, hi
            tris.append((Od[0], Od[1], E[0]))
            tris += [(Od[k], Od[k + 1], E[k]) for k in range(1, n - 1)]
            tris += [(Od[k], E[k], E[k - 1]) for k in range(1, n)]
            tris.append((Od[n - 1], Od[n], E[n - 1]))
    X = np.array(pts, dtype=np.float64)
    height = (ny - 1) * hgt
    tol = 1e-9 * side
    held = (X[:, 0] < tol) | (X[:, 0] > side - tol) | (X[:, 1] < tol) | (X[:, 1] > height - tol)
    return Mesh(f"eqplate{n}", X, np.array(tris, dtype=np.int32), held.astype(np.uint8), model, s,
                dict(n=n, side=side, height=height))


def cylinder_mesh(n: int, radius: float = 0.5, arc: float = math.pi / 4 * 1.0, axial: float = None,
                  jitter: float = 0.0, seed: int = 0, model: str = "FS", pins: str = "ends") -> Mesh:
    """Cylindrical patch of radius R: arc length `arc` around, `axial` along y, n x n vertices.
    pins: 'ends' pins the rows y = 0 and y = axial, 'none' pins nothing."""
    if axial is None:
        axial = arc
    l = arc / (n - 1)
    uv = jitter_uv(grid_uv(n, n, arc, axial), n, n, l, jitter, seed)
    X = cylinder_from_uv(uv, radius, arc / 2.0)
    if pins == "ends":
        pinned = _pins_rows(n, n, [0, n - 1])
    else:
        pinned = np.zeros(n * n, dtype=np.uint8)
    return Mesh(f"cyl{n}", X, grid_tris(n, n), pinned, model, l,
                dict(n=n, radius=radius, arc=arc, axial=axial, jitter=jitter, seed=seed))


def sphere_cap_mesh(n: int, radius: float, side: float = None, jitter: float = 0.0, seed: int = 0,
                    model: str = "SS", pins: str = "ring") -> Mesh:
    """Square of side S (default 1.2 R) lifted onto a sphere of radius R; boundary ring pinned."""
    if side is None:
        side = 1.2 * radius
    l = side / (n - 1)
    uv = jitter_uv(grid_uv(n, n, side, side), n, n, l, jitter, seed)
    X = sphere_cap_from_uv(uv, radius, (side / 2.0, side / 2.0))
    pinned = grid_boundary_mask(n, n).astype(np.uint8) if pins == "ring" else np.zeros(n * n, np.uint8)
    return Mesh(f"cap{n}", X, grid_tris(n, n), pinned, model, l,
                dict(n=n, radius=radius, side=side, jitter=jitter, seed=seed))


def hemisphere_mesh(rings: int = 17, around: int = 64, radius: float = 10.0, cut_deg: float = 18.0,
                    model: str = "SS") -> Mesh:
    """Hemisphere of radius R (pole on +z, equator in z = 0) with a circular hole of half-angle cut_deg
    at the pole: `rings` latitude rings from the hole's rim (ring 0) to the equator, `around` vertices
    per ring starting on +x (vertex id = ring * around + j, azimuth 2 pi j / around), each quad split
    into two triangles.  Nothing pinned."""
    theta = np.radians(np.linspace(cut_deg, 90.0, rings))
    phi = 2.0 * math.pi * np.arange(around) / around
    t, p = np.meshgrid(theta, phi, indexing="ij")
    X = radius * np.stack([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)], axis=-1).reshape(-1, 3)
    # the azimuth grid is closed: column `around` is column 0
    X[np.abs(X) < 1e-12 * radius] = 0.0
    tris = []
    for k in range(rings - 1):
        for j in range(around):
            a, b = k * around + j, k * around + (j + 1) % around
            c, d = a + around, b + around
            tris += [(a, c, d), (a, d, b)]
    return Mesh(f"hemisphere{rings}x{around}", X, np.array(tris, dtype=np.int32),
                np.zeros(rings * around, dtype=np.uint8), model, radius * math.radians(90.0 - cut_deg) / (rings - 1),
                dict(rings=rings, around=around, radius=radius, cut_deg=cut_deg))


HEMISPHERE_MATERIAL = dict(young=6.825e7, poisson=0.3, thickness=0.04, density=1.0)


def hemisphere_problem(rings: int = 17, around: int = 64, load: float = 200.0, model: str = "SS"):
    """The pinched hemisphere with an 18 degree hole: four radial point loads of size `load` on the
    equator, inward on the x axis and outward on the y axis.  Held coordinates: x of the vertices in the
    plane x = 0, y of those in the plane y = 0, and z of the hole-rim vertices in the plane x = 0.
    Returns (mesh, held mask [nv] with bit d holding coordinate d, load [nv, 3], the load vertices on +x
    and +y)."""
    if around % 4:
        raise ValueError("the load points and symmetry planes need around % 4 == 0")
    m = hemisphere_mesh(rings, around, 10.0, 18.0, model)
    j = np.tile(np.arange(around), rings)
    k = np.repeat(np.arange(rings), around)
    q = around // 4
    held = np.zeros(m.nv, dtype=np.uint8)
    held[(j == q) | (j == 3 * q)] |= 1
    held[(j == 0) | (j == 2 * q)] |= 2
    held[(k == 0) & ((j == q) | (j == 3 * q))] |= 4
    F = np.zeros((m.nv, 3))
    eq = (rings - 1) * around
    F[eq + 0, 0] = -load
    F[eq + 2 * q, 0] = load
    F[eq + q, 1] = load
    F[eq + 3 * q, 1] = -load
    return m, held, F, (eq, eq + q)


# --------------------------------------------------------------------------------------------
# The five workloads (shapes, sizes and seeds) that the tests and the benchmark use.
# --------------------------------------------------------------------------------------------

MATERIAL = dict(young=1.0e6, poisson=0.3, thickness=1.0e-3, density=200.0)
GRAVITY = (0.0, 0.0, -9.81)


def workload_plate32() -> Mesh:
    """Flat 1 m square, 32 x 32, edge-hinge plate, one side clamped (x in {0, l} columns pinned)."""
    return plate_mesh(32, 1.0, 0.0, 0, "EP", "clamp_x0")


def workload_cylinder(n: int = 256, model: str = "FS") -> Mesh:
    """Quarter cylinder R = 0.5 (arc and axial length pi/4 * R * 2 = 0.785 m), jitter 0.2 l, pinned ends."""
    arc = 0.5 * math.pi / 2.0
    return cylinder_mesh(n, 0.5, arc, arc, 0.2, 2502108722, model, "ends")


def sphere_cap_radius(seed: int = 2502108723) -> float:
    return float(rng(seed).uniform(0.3, 2.0))


def workload_sphere_cap(n: int = 1024, model: str = "SS") -> Mesh:
    """Sphere cap, R ~ U[0.3, 2] m (seeded), square side 1.2 R, jitter 0.2 l, boundary ring pinned."""
    R = sphere_cap_radius()
    return sphere_cap_mesh(n, R, 1.2 * R, 0.2, 2502108723, model, "ring")


def batch_specs(count: int = 64, seed: int = 2502108724):
    """Mesh specs for the multi-mesh batch: n = round(16 * 32**U), model k mod 6, spacing 1 cm."""
    g = rng(seed)
    specs = []
    for k in range(count):
        n = int(round(16 * 32 ** g.uniform()))
        radius = float(g.uniform(0.3, 2.0))
        sub_seed = int(g.integers(0, 2**31 - 1))
        specs.append(dict(n=n, model=MODELS[k % 6], radius=radius, seed=sub_seed))
    return specs


def mesh_from_spec(spec: dict, spacing: float = 0.01) -> Mesh:
    """Build one batch/serving mesh: plates flat; shells a cylinder (rolled at most to a half turn)
    or a sphere cap when the square fits the cap rule S <= 1.2 R.  Two edge columns pinned."""
    n = spec["n"]
    model = spec["model"]
    side = spacing * (n - 1)
    R = spec["radius"]
    if model.endswith("P"):
        m = plate_mesh(n, side, 0.2, spec["seed"], model, "clamp_x0")
    elif side <= 1.2 * R:
        m = sphere_cap_mesh(n, R, side, 0.2, spec["seed"], model, "ring")
        m.pinned = _pins_columns(n, n, [0, 1])
    else:
        arc = min(side, math.pi * R)
        m = cylinder_mesh(n, R, arc, side, 0.2, spec["seed"], model, "none")
        m.pinned = _pins_columns(n, n, [0, 1])
    m.name = f"{model}{n}"
    return m


def serving_trace(rate: float = 200.0, duration: float = 60.0, seed: int = 2502108725,
                  nv_min: float = 2e3, nv_max: float = 1e6):
    """Poisson arrivals; vertex counts log-normal between nv_min and nv_max (truncated by redraw)."""
    g = rng(seed)
    mu = math.log(math.sqrt(nv_min * nv_max))
    sigma = math.log(nv_max / nv_min) / 6.0 * 1.0
    t = 0.0
    reqs = []
    while True:
        t += g.exponential(1.0 / rate)
        if t > duration:
            break
        while True:
            nv = g.lognormal(mu, sigma)
            if nv_min <= nv <= nv_max:
                break
        n = max(4, int(round(math.sqrt(nv))))
        reqs.append(dict(t=t, n=n, model=MODELS[int(g.integers(0, 6))], radius=float(g.uniform(0.3, 2.0)),
                         seed=int(g.integers(0, 2**31 - 1))))
    return reqs
