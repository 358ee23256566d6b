"""Seeded synthetic inputs for the seeded trajectory optimizer.

This module builds inputs only: the robot description, the box scenes and
their distance grids, seed trajectories and the serving arrival trace.  It
holds none of the optimizer's arithmetic (no kinematics, no cost, no
gradient).  Both the FP64 oracle and the GPU library consume exactly the
float32 arrays produced here.

The paper's workloads (the MpiNet test scenes with a Franka arm, Sec. 5.1)
are not available; these generators stand in for them with the shapes the
method uses: T=32 waypoints of 7 joints (Sec. 4.1), several seeds per
problem (Sec. 5), a signed distance field of the scene (Sec. 4.4), start
configuration and goal pose (Sec. 3).
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 2410167270
N_JOINTS = 7
Q_LIMIT = 2.8


def rng_for(cfg_index: int, *stream: int) -> np.random.Generator:
    """PCG64 stream for config ``cfg_index`` and a sub-stream path."""
    ss = np.random.SeedSequence([BASE_SEED + cfg_index, *stream])
    return np.random.Generator(np.random.PCG64(ss))


# ---------------------------------------------------------------- robot ----

@dataclass
class Robot:
    link_lengths: np.ndarray          # [7] float64 (generation record only)
    frames: np.ndarray                # [8, 12] float32: F_1..F_7, F_ee (3x4 row-major)
    q_lo: np.ndarray                  # [7] float32
    q_hi: np.ndarray                  # [7] float32
    sphere_link: np.ndarray           # [N_s] int32, 1..7
    sphere_offset: np.ndarray         # [N_s, 3] float32, in the link frame
    sphere_radius: np.ndarray         # [N_s] float32

    @property
    def n_spheres(self) -> int:
        return int(self.sphere_link.shape[0])


def _frame(R, p) -> np.ndarray:
    out = np.zeros(12, dtype=np.float32)
    out[0:3] = R[0]
    out[4:7] = R[1]
    out[8:11] = R[2]
    out[3], out[7], out[11] = p
    return out


def make_robot(rng_links: np.random.Generator, rng_spheres: np.random.Generator,
               spheres_per_link) -> Robot:
    """Synthetic 7-revolute serial arm.

    Link lengths U[0.08, 0.35] m, joint limits +-2.8 rad.  Joint i (1-based)
    rotates about its local z axis.  The fixed transform before joint 1 is
    the identity; before joint i>1 it is a translation of L_{i-1} along z
    followed by a twist of -pi/2 (even i) or +pi/2 (odd i) about x.  The
    end-effector frame sits L_7 along z of link 7.  Link l carries
    ``spheres_per_link[l-1]`` spheres evenly spaced on its z segment with
    radii U[0.03, 0.08] m.  The twist matrices are written with exact
    0/+-1 entries.  Link lengths and sphere radii come from separate
    streams so that every workload shares one arm.
    """
    L = rng_links.uniform(0.08, 0.35, size=N_JOINTS)
    rx_plus = [[1, 0, 0], [0, 0, -1], [0, 1, 0]]    # Rx(+pi/2)
    rx_minus = [[1, 0, 0], [0, 0, 1], [0, -1, 0]]   # Rx(-pi/2)
    frames = np.zeros((8, 12), dtype=np.float32)
    frames[0] = _frame(np.eye(3), (0.0, 0.0, 0.0))
    for i in range(2, N_JOINTS + 1):
        R = rx_minus if i % 2 == 0 else rx_plus
        frames[i - 1] = _frame(np.array(R, dtype=np.float64), (0.0, 0.0, L[i - 2]))
    frames[7] = _frame(np.eye(3), (0.0, 0.0, L[6]))
    links, offs, rads = [], [], []
    for l in range(1, N_JOINTS + 1):
        n = int(spheres_per_link[l - 1])
        for k in range(n):
            links.append(l)
            offs.append((0.0, 0.0, (k + 0.5) * L[l - 1] / n))
            rads.append(rng_spheres.uniform(0.03, 0.08))
    return Robot(
        link_lengths=L,
        frames=frames,
        q_lo=np.full(N_JOINTS, -Q_LIMIT, dtype=np.float32),
        q_hi=np.full(N_JOINTS, Q_LIMIT, dtype=np.float32),
        sphere_link=np.array(links, dtype=np.int32),
        sphere_offset=np.array(offs, dtype=np.float32),
        sphere_radius=np.array(rads, dtype=np.float32),
    )


# ---------------------------------------------------------------- scenes ---

@dataclass
class Scene:
    box_centre: np.ndarray            # [B, 3] float64
    box_half: np.ndarray              # [B, 3] float64
    dims: tuple                       # (nx, ny, nz)
    voxel: float
    origin: np.ndarray                # [3] float32
    grid: np.ndarray | None = field(default=None, repr=False)  # [nz, ny, nx] float32 (x fastest)

    @property
    def hi(self) -> np.ndarray:
        return self.origin.astype(np.float64) + (np.array(self.dims) - 1) * self.voxel


def f32(v) -> float:
    """The float32 value of ``v`` (grid spacing and origin are float32 at
    the library boundary; node positions use exactly those values)."""
    return float(np.float32(v))


MARGIN = 0.02 + 0.08 + 0.005   # activation distance + largest radius + slack
BASE_KEEPOUT = 0.25             # xy distance of every random box from the base axis


def box_sdf(points: np.ndarray, centre: np.ndarray, half: np.ndarray) -> np.ndarray:
    """Signed distance (negative inside) from ``points`` [..., 3] to one
    axis-aligned box, FP64."""
    q = np.abs(points - centre) - half
    outside = np.sqrt(np.sum(np.maximum(q, 0.0) ** 2, axis=-1))
    inside = np.minimum(np.max(q, axis=-1), 0.0)
    return outside + inside


def scene_sdf(points: np.ndarray, scene: Scene) -> np.ndarray:
    d = np.full(points.shape[:-1], np.inf)
    for c, h in zip(scene.box_centre, scene.box_half):
        d = np.minimum(d, box_sdf(points, c, h))
    return d


def _grid_slab(scene: Scene, k0: int, k1: int) -> np.ndarray:
    """Exact scene distance on the node slab k0 <= k < k1, using the
    per-axis split of the box distance (the same sum order as
    ``box_sdf``)."""
    nx, ny, nz = scene.dims
    o = scene.origin.astype(np.float64)
    xs = o[0] + np.arange(nx) * scene.voxel
    ys = o[1] + np.arange(ny) * scene.voxel
    zs = o[2] + np.arange(k0, k1) * scene.voxel
    d = np.full((k1 - k0, ny, nx), np.inf)
    tmp = np.empty_like(d)
    ins = np.empty_like(d)
    for c, h in zip(scene.box_centre, scene.box_half):
        qx = np.abs(xs - c[0]) - h[0]
        qy = np.abs(ys - c[1]) - h[1]
        qz = np.abs(zs - c[2]) - h[2]
        ax = np.maximum(qx, 0.0) ** 2
        ay = np.maximum(qy, 0.0) ** 2
        az = np.maximum(qz, 0.0) ** 2
        np.add(ax[None, None, :], ay[None, :, None], out=tmp)
        np.add(tmp, az[:, None, None], out=tmp)
        np.sqrt(tmp, out=tmp)
        np.maximum(qx[None, None, :], qy[None, :, None], out=ins)
        np.maximum(ins, qz[:, None, None], out=ins)
        np.minimum(ins, 0.0, out=ins)
        np.add(tmp, ins, out=tmp)
        np.minimum(d, tmp, out=d)
    return d.astype(np.float32)


def build_grid(scene: Scene, threads: int = 8) -> np.ndarray:
    """Node-centred grid of the exact scene distance, x fastest, FP64
    evaluated, stored FP32.  Nodes sit at origin + (i, j, k) * voxel."""
    nx, ny, nz = scene.dims
    step = max(1, (nz + 4 * threads - 1) // (4 * threads))
    slabs = [(k, min(nz, k + step)) for k in range(0, nz, step)]
    out = np.empty((nz, ny, nx), dtype=np.float32)
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        for (k0, k1), part in zip(slabs, ex.map(lambda s: _grid_slab(scene, *s), slabs)):
            out[k0:k1] = part
    return out


def _fit_box(rng, lo, hi, extent, annulus=None, tries=200):
    """Place a box of full size ``extent`` fully inside [lo, hi]; with an
    annulus (rmin, rmax) its xy centre radius is constrained."""
    half = np.minimum(extent / 2.0, (hi - lo) / 2.0 - 1e-3)
    for _ in range(tries):
        c = rng.uniform(lo + half, hi - half)
        if annulus is not None:
            r = math.hypot(c[0], c[1])
            if not (annulus[0] <= r <= annulus[1]):
                continue
            # keep the base column (the first link never moves) free
            gx = max(abs(c[0]) - half[0], 0.0)
            gy = max(abs(c[1]) - half[1], 0.0)
            if math.hypot(gx, gy) < BASE_KEEPOUT:
                continue
        return c, half
    return None


def random_box_scene(rng, n_boxes, dims, voxel, origin, annulus=(0.3, 0.75)) -> Scene:
    origin = np.asarray(origin, dtype=np.float32)
    sc = Scene(np.zeros((0, 3)), np.zeros((0, 3)), tuple(dims), f32(voxel), origin)
    lo = sc.origin.astype(np.float64) + MARGIN
    hi = sc.hi - MARGIN
    cs, hs = [], []
    while len(cs) < n_boxes:
        ext = rng.uniform(0.02, 0.6, size=3)
        placed = _fit_box(rng, lo, hi, ext, annulus)
        if placed is None:
            continue
        cs.append(placed[0])
        hs.append(placed[1])
    sc.box_centre = np.array(cs)
    sc.box_half = np.array(hs)
    return sc


def shelf_scene(rng, n_boxes, dims, voxel, origin) -> Scene:
    """Shelf layout: 2-3 bays 0.4-0.9 m from the base, each with two side
    panels, a back panel and two shelves (thin boxes, thin extent
    U[0.02, 0.04]); the remaining boxes are clutter placed in the bays
    (extents U[0.02, 0.6] clipped to the bay interior)."""
    origin = np.asarray(origin, dtype=np.float32)
    sc = Scene(np.zeros((0, 3)), np.zeros((0, 3)), tuple(dims), f32(voxel), origin)
    glo = sc.origin.astype(np.float64) + MARGIN
    ghi = sc.hi - MARGIN
    n_bays = int(rng.integers(2, 4))
    dirs = rng.permutation(4)[:n_bays]            # +x, +y, -x, -y
    cs, hs, interiors = [], [], []
    for b in dirs:
        width = rng.uniform(0.3, 0.6)
        depth = rng.uniform(0.2, 0.4)
        height = rng.uniform(0.4, 0.6)
        t = lambda: rng.uniform(0.02, 0.04)
        near = rng.uniform(0.4, 0.9 - depth)
        far = near + depth
        lat = rng.uniform(-0.2, 0.2)
        z0 = rng.uniform(0.0, 0.3)
        # box in bay-local coordinates (u = outward, v = lateral, z)
        local = []
        ts = t()
        local.append(((near + far) / 2, lat - width / 2, z0 + height / 2, depth / 2, ts / 2, height / 2))
        ts = t()
        local.append(((near + far) / 2, lat + width / 2, z0 + height / 2, depth / 2, ts / 2, height / 2))
        ts = t()
        local.append((far, lat, z0 + height / 2, ts / 2, width / 2, height / 2))
        ts = t()
        local.append(((near + far) / 2, lat, z0, depth / 2, width / 2, ts / 2))
        ts = t()
        local.append(((near + far) / 2, lat, z0 + height / 2, depth / 2, width / 2, ts / 2))
        for (u, v, z, hu, hv, hz) in local:
            c, h = _bay_to_world(b, u, v, z, hu, hv, hz)
            cs.append(c)
            hs.append(h)
        interiors.append((b, near, far, lat - width / 2, lat + width / 2, z0, z0 + height))
    while len(cs) < n_boxes:
        b, near, far, v0, v1, z0, z1 = interiors[int(rng.integers(len(interiors)))]
        ext = rng.uniform(0.02, 0.6, size=3)
        hu = min(ext[0], far - near - 0.08) / 2
        hv = min(ext[1], v1 - v0 - 0.08) / 2
        hz = min(ext[2], (z1 - z0) / 2 - 0.04) / 2
        u = rng.uniform(near + 0.03 + hu, far - 0.03 - hu)
        v = rng.uniform(v0 + 0.03 + hv, v1 - 0.03 - hv)
        z = z0 + 0.02 + hz
        c, h = _bay_to_world(b, u, v, z, hu, hv, hz)
        cs.append(c)
        hs.append(h)
    cs = np.array(cs)
    hs = np.array(hs)
    # keep every box inside the grid with the clamp margin
    lo_c = np.maximum(cs - hs, glo)
    hi_c = np.minimum(cs + hs, ghi)
    sc.box_centre = (lo_c + hi_c) / 2
    sc.box_half = np.maximum((hi_c - lo_c) / 2, 0.005)
    return sc


def _bay_to_world(b, u, v, z, hu, hv, hz):
    if b == 0:
        return np.array([u, v, z]), np.array([hu, hv, hz])
    if b == 1:
        return np.array([-v, u, z]), np.array([hv, hu, hz])
    if b == 2:
        return np.array([-u, -v, z]), np.array([hu, hv, hz])
    return np.array([v, -u, z]), np.array([hv, hu, hz])


def build_grids(scenes, threads: int = 8):
    """Fill ``scene.grid`` for every scene that has none."""
    for s in scenes:
        if s.grid is None:
            s.grid = build_grid(s, threads)
    return scenes


def occupancy(scene: Scene) -> np.ndarray:
    """Occupancy of the grid nodes (uint8 [nz, ny, nx]): 1 where the node
    lies strictly inside a box.  Input for building the distance field on
    the GPU."""
    if scene.grid is not None:
        return (scene.grid < 0).astype(np.uint8)
    g = build_grid(scene)
    return (g < 0).astype(np.uint8)


def empty_scene(dims=(16, 16, 16), voxel=0.2, origin=(-1.6, -1.6, -1.6), value=1.0) -> Scene:
    sc = Scene(np.zeros((0, 3)), np.zeros((0, 3)), tuple(dims), f32(voxel),
               np.asarray(origin, dtype=np.float32))
    sc.grid = np.full(dims[::-1], value, dtype=np.float32)
    return sc


# ----------------------------------------------------------------- seeds ---

def interp_seeds(rng, q_start, q_goal, S, T, sigma=0.1, q_lo=-Q_LIMIT, q_hi=Q_LIMIT) -> np.ndarray:
    """Seeds [S, T, 7] float32: linear interpolation from q_start to q_goal
    plus N(0, sigma) on waypoints 1..T-1, clipped to the joint limits.
    Waypoint 0 equals q_start.  Stands in for the diffusion seeder's
    output (Sec. 4.3)."""
    q_start = np.asarray(q_start, dtype=np.float64)
    q_goal = np.asarray(q_goal, dtype=np.float64)
    a = np.linspace(0.0, 1.0, T)[:, None]
    base = (1.0 - a) * q_start[None, :] + a * q_goal[None, :]
    seeds = np.repeat(base[None], S, axis=0)
    seeds[:, 1:, :] += rng.normal(0.0, sigma, size=(S, T - 1, N_JOINTS))
    seeds = np.clip(seeds, q_lo, q_hi)
    seeds[:, 0, :] = q_start
    return seeds.astype(np.float32)


def random_trajectories(rng, S, T, q_start=None, scale=1.0) -> np.ndarray:
    """Arbitrary trajectories inside the limits (for cost/gradient tests)."""
    X = rng.uniform(-Q_LIMIT * scale, Q_LIMIT * scale, size=(S, T, N_JOINTS))
    if q_start is not None:
        X[:, 0, :] = q_start
    return X.astype(np.float32)


def poisson_arrivals(rng, n, rate_hz) -> np.ndarray:
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
