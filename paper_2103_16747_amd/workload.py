"""Seeded synthetic inputs for the indentation solves: tetrahedral meshes,
Dirichlet masks and indenter load schedules.

The paper's own meshes and indentation records are not available (its BioTac
skin mesh is built from a commercial model, Sec. III-A; its indentation set is
re-simulated lab data, Sec. III-C), so every input here is synthetic with the
paper's workload shape: a soft skin shell bonded to a rigid core, clamped on
its base, indented by rigid spheres, cylinders, boxes and rings (the indenter
families named in Sec. IV-A and Fig. 5) at random surface points and depths.

This module is shared by the device path, the CPU oracle and the benchmarks,
so it deliberately holds no part of the solve: no deformation gradients,
stresses, signed distances or contact arithmetic. It only produces integers,
coordinates, masks and poses. All randomness comes from xoshiro256** seeded
through SplitMix64 (Blackman and Vigna, "Scrambled linear pseudorandom number
generators", 2021), implemented here from its published definition.

Units are SI throughout (metres, pascals, newtons).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1

# Indenter kinds (match the C ABI's numbering).
SPHERE, CYLINDER, BOX, RING = 0, 1, 2, 3
KIND_NAMES = {SPHERE: "sphere", CYLINDER: "cylinder", BOX: "box", RING: "ring"}


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------
def _rotl(x: int, k: int) -> int:
    return ((x << k) | (x >> (64 - k))) & MASK64


class Xoshiro256ss:
    """xoshiro256** with its state filled by SplitMix64 from one 64-bit seed."""

    def __init__(self, seed: int):
        s = seed & MASK64
        st = []
        for _ in range(4):
            s = (s + 0x9E3779B97F4A7C15) & MASK64
            z = s
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
            st.append(z ^ (z >> 31))
        self.s = st

    def next_u64(self) -> int:
        s = self.s
        result = (_rotl((s[1] * 5) & MASK64, 7) * 9) & MASK64
        t = (s[1] << 17) & MASK64
        s[2] ^= s[0]
        s[3] ^= s[1]
        s[1] ^= s[2]
        s[0] ^= s[3]
        s[2] ^= t
        s[3] = _rotl(s[3], 45)
        return result

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        """Double in [lo, hi) from the top 53 bits."""
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def below(self, n: int) -> int:
        """Integer in [0, n) (n small; the modulo bias is below 2^-50)."""
        return self.next_u64() % n


def instance_seed(config: int, instance: int) -> int:
    """Seed of instance `instance` of workload family `config` (1-based)."""
    return 1000 * config + instance


# --------------------------------------------------------------------------
# Meshes
# --------------------------------------------------------------------------
# The six tetrahedra of the Kuhn (Freudenthal) split of a cell, one per axis
# order (a, b, c): {v, v+e_a, v+e_a+e_b, v+e_a+e_b+e_c}. Corners are numbered
# by bits (x=1, y=2, z=4). The signed volume of such a tet on a box with
# positive extents has the sign of the permutation, so odd orders swap their
# second and third vertex to keep every tet positively oriented.
def _kuhn_local():
    out = []
    for perm in ((0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)):
        even = perm in ((0, 1, 2), (1, 2, 0), (2, 0, 1))
        a, b, c = perm
        v0 = 0
        v1 = v0 | (1 << a)
        v2 = v1 | (1 << b)
        v3 = v2 | (1 << c)
        out.append((v0, v1, v2, v3) if even else (v0, v2, v1, v3))
    return np.array(out, dtype=np.int64)


KUHN_LOCAL = _kuhn_local()


@dataclass
class Mesh:
    """A linear-tetrahedron mesh with a Dirichlet mask.

    X: (n, 3) float64 rest positions; tets: (m, 4) int32, positively oriented;
    fixed: (n,) uint8, 1 where the node's displacement is prescribed.
    """
    X: np.ndarray
    tets: np.ndarray
    fixed: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def m(self) -> int:
        return int(self.tets.shape[0])


def _voxel_mesh(xs, ys, zs, keep):
    """Kuhn-split every kept cell of the tensor grid (xs, ys, zs).

    keep: bool array (len(xs)-1, len(ys)-1, len(zs)-1). Returns (X, tets,
    node_grid_index) with only the nodes used by kept cells, numbered in
    (z, y, x)-lexicographic grid order, and tets in cell order.
    """
    nx, ny, nz = len(xs), len(ys), len(zs)
    ci, cj, ck = np.nonzero(keep)
    order = np.lexsort((ci, cj, ck))          # cells in (z, y, x) order
    ci, cj, ck = ci[order], cj[order], ck[order]
    corner = np.empty((len(ci), 8), dtype=np.int64)
    for bits in range(8):
        dx, dy, dz = bits & 1, (bits >> 1) & 1, (bits >> 2) & 1
        corner[:, bits] = ((ck + dz) * ny + (cj + dy)) * nx + (ci + dx)
    tets_grid = corner[:, KUHN_LOCAL].reshape(-1, 4)
    used = np.unique(tets_grid)
    remap = np.full(nx * ny * nz, -1, dtype=np.int64)
    remap[used] = np.arange(len(used))
    gi = used % nx
    gj = (used // nx) % ny
    gk = used // (nx * ny)
    X = np.stack([np.asarray(xs)[gi], np.asarray(ys)[gj], np.asarray(zs)[gk]], axis=1)
    return X.astype(np.float64), remap[tets_grid].astype(np.int32), used, remap


def block_mesh(cells=(8, 8, 8), size=(0.01, 0.01, 0.01), xs=None, ys=None, zs=None) -> Mesh:
    """Rectangular elastomer block, Kuhn-split, base (z = z_min) clamped.

    With explicit coordinate arrays xs/ys/zs the grid may be graded.
    """
    if xs is None:
        xs = np.linspace(0.0, size[0], cells[0] + 1)
    if ys is None:
        ys = np.linspace(0.0, size[1], cells[1] + 1)
    if zs is None:
        zs = np.linspace(0.0, size[2], cells[2] + 1)
    keep = np.ones((len(xs) - 1, len(ys) - 1, len(zs) - 1), dtype=bool)
    X, tets, _, _ = _voxel_mesh(xs, ys, zs, keep)
    fixed = (X[:, 2] == zs[0]).astype(np.uint8)
    return Mesh(X, tets, fixed, name="block")


def cube_block_mesh() -> Mesh:
    """Single elastomer block: 8x8x8 cells over a 10 mm cube, 3072 tets and
    729 nodes, bottom face fixed."""
    m = block_mesh((8, 8, 8), (0.01, 0.01, 0.01))
    m.name = "cube8"
    return m


# Fingertip design geometry (mm): a cylindrical shell of outer radius 7 and
# inner radius 4 from z = 0 to 30, capped by half-spheroids with axial
# semi-axes 10 (outer) and 7 (inner): 40 mm long and 3 mm thick.
FT_R_OUT, FT_R_IN = 7.0e-3, 4.0e-3
FT_L_CYL = 30.0e-3
FT_C_OUT, FT_C_IN = 10.0e-3, 7.0e-3

# Voxel sizes that give about 5k / 20k / 50k / 120k tets.
FINGERTIP_VOXEL = {5000: 1.646e-3, 20000: 1.060e-3, 50000: 0.772e-3, 120000: 0.581e-3}


def _in_capsule(x, y, z, R, c):
    rho2 = x * x + y * y
    cyl = (z >= 0.0) & (z <= FT_L_CYL) & (rho2 <= R * R)
    cap = (z > FT_L_CYL) & (rho2 / (R * R) + ((z - FT_L_CYL) / c) ** 2 <= 1.0)
    return cyl | cap


def fingertip_mesh(target_tets: int = 50000, h: float | None = None) -> Mesh:
    """Synthetic fingertip: voxel-Kuhn mesh of the skin shell around a rigid core.

    A cell is kept when its centre lies in the shell (inside the outer capsule,
    outside the inner one). Fixed nodes are the corners of cells whose centre
    lies in the inner capsule (the skin is bonded to the rigid core over its
    whole inner surface) and the nodes on the base plane z = 0 (the clamp).
    """
    if h is None:
        h = FINGERTIP_VOXEL[target_tets]
    nxc = int(math.ceil(2 * FT_R_OUT / h)) + 2
    nxc += nxc % 2
    nzc = int(math.ceil((FT_L_CYL + FT_C_OUT) / h)) + 1
    xs = (np.arange(nxc + 1) - nxc / 2) * h
    zs = np.arange(nzc + 1) * h
    cx = 0.5 * (xs[:-1] + xs[1:])
    cz = 0.5 * (zs[:-1] + zs[1:])
    CX, CY, CZ = np.meshgrid(cx, cx, cz, indexing="ij")
    outer = _in_capsule(CX, CY, CZ, FT_R_OUT, FT_C_OUT)
    inner = _in_capsule(CX, CY, CZ, FT_R_IN, FT_C_IN)
    keep = outer & ~inner
    X, tets, used, remap = _voxel_mesh(xs, xs, zs, keep)
    # Corners of core cells -> bonded to the rigid core.
    nx = ny = len(xs)
    ci, cj, ck = np.nonzero(inner)
    core_nodes = []
    for bits in range(8):
        dx, dy, dz = bits & 1, (bits >> 1) & 1, (bits >> 2) & 1
        core_nodes.append(((ck + dz) * ny + (cj + dy)) * nx + (ci + dx))
    core_nodes = np.unique(np.concatenate(core_nodes))
    fixed = np.zeros(len(used), dtype=np.uint8)
    idx = remap[core_nodes]
    fixed[idx[idx >= 0]] = 1
    fixed[X[:, 2] == 0.0] = 1
    return Mesh(X, tets, fixed, name=f"fingertip{target_tets // 1000}k", meta={"h": h})


# --------------------------------------------------------------------------
# Indenters and load schedules
# --------------------------------------------------------------------------
@dataclass
class Indentation:
    """A rigid indenter pressed along `direction` in `steps` equal increments.

    kind/shape follow the C ABI: sphere (r), cylinder (radius, height), box
    (half extents), ring (major radius, minor radius). R's third column is the
    indenter's local axis; the indenter's leading point (or leading face or
    circle) touches the design surface at contact_point when the depth is 0.
    """
    kind: int
    shape: np.ndarray
    R: np.ndarray
    c0: np.ndarray
    direction: np.ndarray
    depth: float
    steps: int
    k_penalty: float = 1.0e4
    contact_point: np.ndarray | None = None
    seed: int | None = None
    dt: float = 0.0           # > 0: implicit time steps of this length (s)
    density: float = 1100.0   # kg/m^3, lumped masses of implicit steps
    model: int = 0            # 0 Neo-Hookean, 1 co-rotational linear elasticity
    friction: float = 0.0     # Coulomb coefficient (0: frictionless)
    friction_eps: float = 1e-5  # slip smoothing length (m)

    def center(self, step: int) -> np.ndarray:
        """Indenter centre at load step `step` (0 = initial contact pose)."""
        return self.c0 + (self.depth * step / self.steps) * self.direction

    def poses(self):
        return [(self.R, self.center(k)) for k in range(1, self.steps + 1)]


def cube_sphere_indentation(steps: int = 10, depth: float = 1.5e-3) -> Indentation:
    """Sphere of radius 3 mm pressed centrally into the top of the 10 mm block,
    1.5 mm in 10 steps (centre at z = 13 - 0.15 k mm)."""
    return Indentation(SPHERE, np.array([3.0e-3]), np.eye(3), np.array([5e-3, 5e-3, 13e-3]),
                       np.array([0.0, 0.0, -1.0]), depth, steps)


def _frame_from_axis(axis: np.ndarray, yaw: float = 0.0) -> np.ndarray:
    """Orthonormal matrix whose third column is `axis`, first two turned by yaw."""
    a = axis / np.linalg.norm(axis)
    helper = np.array([1.0, 0.0, 0.0]) if abs(a[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t1 = np.cross(a, helper)
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(a, t1)
    cy, sy = math.cos(yaw), math.sin(yaw)
    e1 = cy * t1 + sy * t2
    e2 = -sy * t1 + cy * t2
    return np.stack([e1, e2, a], axis=1)


def _sample_fingertip_surface(rng: Xoshiro256ss, zmin: float = 5.0e-3):
    """Point and outward normal, uniform by area over the outer design surface
    with z >= zmin (cylinder side plus the half-spheroid cap)."""
    a, c = FT_R_OUT, FT_C_OUT
    area_cyl = 2 * math.pi * a * (FT_L_CYL - zmin)
    # Prolate half-spheroid area: pi a^2 + pi a c asin(e) / e, halved.
    e = math.sqrt(1.0 - (a * a) / (c * c))
    area_cap = 0.5 * (2 * math.pi * a * a + 2 * math.pi * a * c * math.asin(e) / e)
    if rng.uniform() < area_cyl / (area_cyl + area_cap):
        th = rng.uniform(0.0, 2 * math.pi)
        z = rng.uniform(zmin, FT_L_CYL)
        n = np.array([math.cos(th), math.sin(th), 0.0])
        p = np.array([a * n[0], a * n[1], z])
        return p, n
    # Cap: map uniform points of the upper unit hemisphere onto the spheroid,
    # accepted with probability proportional to the area stretch.
    while True:
        w = rng.uniform()
        th = rng.uniform(0.0, 2 * math.pi)
        s = math.sqrt(max(0.0, 1.0 - w * w))
        u, v = s * math.cos(th), s * math.sin(th)
        stretch = a * math.sqrt(c * c * (u * u + v * v) + a * a * w * w)
        if rng.uniform() * (a * max(a, c)) <= stretch:
            p = np.array([a * u, a * v, FT_L_CYL + c * w])
            n = np.array([p[0] / (a * a), p[1] / (a * a), (p[2] - FT_L_CYL) / (c * c)])
            return p, n / np.linalg.norm(n)


def random_indentation(seed: int, steps: int = 100, max_depth: float = 3.0e-3,
                       k_penalty: float = 1.0e4) -> Indentation:
    """One seeded indentation of the fingertip.

    Draw order: kind; shape parameters; surface point; tilt cos(theta) in
    [cos 30 deg, 1] and azimuth; yaw (box only); depth in [0, max_depth].
    """
    rng = Xoshiro256ss(seed)
    kind = rng.below(4)
    if kind == SPHERE:
        shape = np.array([rng.uniform(2e-3, 6e-3)])
        lead = shape[0]
    elif kind == CYLINDER:
        shape = np.array([rng.uniform(1.5e-3, 4e-3), 5e-3])
        lead = 0.5 * shape[1]
    elif kind == BOX:
        shape = np.array([rng.uniform(1e-3, 4e-3), rng.uniform(1e-3, 4e-3), rng.uniform(1e-3, 4e-3)])
        lead = shape[2]
    else:
        shape = np.array([rng.uniform(3e-3, 5e-3), rng.uniform(0.5e-3, 1.5e-3)])
        lead = shape[1]
    p, nrm = _sample_fingertip_surface(rng)
    cos_t = rng.uniform(math.cos(math.radians(30.0)), 1.0)
    sin_t = math.sqrt(max(0.0, 1.0 - cos_t * cos_t))
    az = rng.uniform(0.0, 2 * math.pi)
    F = _frame_from_axis(nrm)
    d = -cos_t * nrm + sin_t * (math.cos(az) * F[:, 0] + math.sin(az) * F[:, 1])
    d /= np.linalg.norm(d)
    yaw = rng.uniform(0.0, 2 * math.pi) if kind == BOX else 0.0
    depth = rng.uniform(0.0, max_depth)
    R = _frame_from_axis(d, yaw)
    c0 = p - lead * d
    return Indentation(kind, shape, R, c0, d, depth, steps, k_penalty, contact_point=p, seed=seed)


# --------------------------------------------------------------------------
# Seating: depth is measured from the pose of initial contact (Fig. 2 caption)
# --------------------------------------------------------------------------
def _interval_quadratic(a2, a1, a0):
    """t-interval where a2 t^2 + a1 t + a0 <= 0 (a2 >= 0), vectorised.
    Returns (lo, hi) with lo > hi marking an empty interval."""
    lo = np.full(a0.shape, np.inf)
    hi = np.full(a0.shape, -np.inf)
    quad = a2 > 1e-300
    disc = a1 * a1 - 4.0 * a2 * a0
    ok = quad & (disc >= 0.0)
    sq = np.sqrt(np.where(ok, disc, 0.0))
    lo = np.where(ok, (-a1 - sq) / np.where(quad, 2.0 * a2, 1.0), lo)
    hi = np.where(ok, (-a1 + sq) / np.where(quad, 2.0 * a2, 1.0), hi)
    const = ~quad & (a0 <= 0.0)
    lo = np.where(const, -np.inf, lo)
    hi = np.where(const, np.inf, hi)
    return lo, hi


def _slab(a, d, half):
    """t-interval where |a - t d| <= half, vectorised over a."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (a - half) / d
        t2 = (a + half) / d
    lo = np.where(d != 0.0, np.minimum(t1, t2), np.where(np.abs(a) <= half, -np.inf, np.inf))
    hi = np.where(d != 0.0, np.maximum(t1, t2), np.where(np.abs(a) <= half, np.inf, -np.inf))
    return lo, hi


def first_contact_shift(ind: Indentation, points: np.ndarray) -> float:
    """Smallest translation t along ind.direction at which the indenter, placed
    at c0 + t d, first touches one of `points` (ray casting in the indenter's
    frame; the ring is root-bracketed on a fine grid and bisected)."""
    a = (points - ind.c0) @ ind.R           # local coordinates at t = 0
    dl = ind.R.T @ ind.direction            # a point moves by -t dl
    if ind.kind == SPHERE:
        r = ind.shape[0]
        lo, hi = _interval_quadratic(np.full(len(a), dl @ dl), -2.0 * (a @ dl), np.einsum("ij,ij->i", a, a) - r * r)
    elif ind.kind == BOX:
        lo, hi = np.full(len(a), -np.inf), np.full(len(a), np.inf)
        for i in range(3):
            l2, h2 = _slab(a[:, i], np.full(len(a), dl[i]), ind.shape[i])
            lo, hi = np.maximum(lo, l2), np.minimum(hi, h2)
    elif ind.kind == CYLINDER:
        rad, hh = ind.shape[0], 0.5 * ind.shape[1]
        dxy = dl[:2]
        l1, h1 = _interval_quadratic(np.full(len(a), dxy @ dxy), -2.0 * (a[:, :2] @ dxy),
                                     np.einsum("ij,ij->i", a[:, :2], a[:, :2]) - rad * rad)
        l2, h2 = _slab(a[:, 2], np.full(len(a), dl[2]), hh)
        lo, hi = np.maximum(l1, l2), np.minimum(h1, h2)
    else:
        Rm, rm = ind.shape[0], ind.shape[1]

        def inside(pts, t):
            p = pts - t[..., None] * dl
            rho = np.sqrt(p[..., 0] ** 2 + p[..., 1] ** 2)
            return (rho - Rm) ** 2 + p[..., 2] ** 2 - rm * rm <= 0.0

        # Only points whose ray passes within the bounding sphere can be hit.
        l0, h0 = _interval_quadratic(np.full(len(a), dl @ dl), -2.0 * (a @ dl),
                                     np.einsum("ij,ij->i", a, a) - (Rm + rm) ** 2)
        cand = np.nonzero(l0 <= h0)[0]
        lo = np.full(len(a), np.inf)
        hi = np.full(len(a), -np.inf)
        if len(cand):
            ac = a[cand]
            step = rm / 16.0
            nsamp = int(np.ceil((h0[cand] - l0[cand]).max() / step)) + 2
            ts = l0[cand][:, None] + step * np.arange(nsamp)[None, :]
            ins = inside(ac[:, None, :], ts) & (ts <= h0[cand][:, None])
            hit = np.nonzero(ins.any(axis=1))[0]
            first = np.argmax(ins, axis=1)[hit]
            t_in = ts[hit, first]
            t_out = np.where(first > 0, ts[hit, np.maximum(first - 1, 0)], l0[cand][hit])
            for _ in range(60):
                mid = 0.5 * (t_in + t_out)
                sel = inside(ac[hit], mid)
                t_in = np.where(sel, mid, t_in)
                t_out = np.where(sel, t_out, mid)
            lo[cand[hit]] = t_in
            hi[cand[hit]] = t_in
    valid = lo <= hi
    if not valid.any():
        raise ValueError("indenter path misses every point")
    return float(lo[valid].min())


def seat_on_mesh(ind: Indentation, mesh: Mesh) -> Indentation:
    """Moves c0 along the press direction to the pose of first contact with the
    mesh's free nodes, so that no node penetrates at depth 0 and one touches."""
    pts = mesh.X[mesh.fixed == 0]
    t = first_contact_shift(ind, pts)
    out = Indentation(ind.kind, ind.shape.copy(), ind.R.copy(), ind.c0 + t * ind.direction, ind.direction.copy(),
                      ind.depth, ind.steps, ind.k_penalty, contact_point=ind.contact_point, seed=ind.seed)
    return out


def poisson_arrivals(seed: int, rate: float, count: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream with the given rate."""
    rng = Xoshiro256ss(seed)
    t, out = 0.0, np.empty(count)
    for i in range(count):
        t += -math.log(1.0 - rng.uniform()) / rate
        out[i] = t
    return out


def random_displacement(mesh: Mesh, seed: int, scale: float) -> np.ndarray:
    """Seeded smooth-plus-noise displacement field (zero on fixed nodes), used
    as an arbitrary state at which single evaluations are compared."""
    rng = Xoshiro256ss(seed)
    coef = np.array([rng.uniform(-1, 1) for _ in range(12)])
    X = mesh.X
    L = np.ptp(X, axis=0).max()
    xi = (X - X.min(axis=0)) / L
    u = np.empty_like(X)
    for d in range(3):
        a, b, c, e = coef[4 * d: 4 * d + 4]
        u[:, d] = a * np.sin(3.0 * xi[:, 0] + b) * np.cos(2.0 * xi[:, 1] + c) * xi[:, 2] + e * xi[:, 2] ** 2
    noise_rng = np.random.Generator(np.random.PCG64(seed))
    u += 0.05 * noise_rng.uniform(-1.0, 1.0, size=u.shape)
    u *= scale * L
    u[mesh.fixed.astype(bool)] = 0.0
    return u
