"""Seeded synthetic triangle meshes used as inputs by both the GPU path and the oracle.

This module builds geometry only; it contains none of the embedding arithmetic
(classification, refinement, cut links).  Every mesh is closed, oriented with
outward normals (counter-clockwise seen from outside) and non-self-intersecting,
which is the input contract of the method (Methodology, "Overview", and the
assumptions listed under "Voxelization and Near-Wall Refinement").

Coordinates are in base-cell units: the domain is [0, N]^3 with unit base cells.

The paper measures on the Stanford bunny (112,394 triangles) and the XYZ RGB
dragon (7,218,906 triangles) (Table 1).  Those scans are not available here;
the lat-long "star" meshes below stand in for them with the same triangle
counts (112,000 and 7,200,000) and a noisy, locally concave/convex surface.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import lpmv


@dataclass
class Mesh:
    verts: np.ndarray          # [nv, 3] float64 or float32
    tris: np.ndarray           # [nt, 3] int32, outward CCW
    name: str = "mesh"
    meta: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return int(self.verts.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tris.shape[0])


# ----------------------------------------------------------------------------
# icosphere
# ----------------------------------------------------------------------------

def icosphere(subdivisions: int = 3, radius: float = 12.0,
              centre=(32.3, 31.7, 32.1)) -> Mesh:
    """Icosahedron refined by midpoint subdivision, midpoints projected onto the
    sphere in float64.  3 subdivisions give 20*4^3 = 1,280 triangles and 642
    vertices."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-phi, phi):
            v.append((0.0, s1, s2))
            v.append((s1, s2, 0.0))
            v.append((s2, 0.0, s1))
    verts = [np.array(p) / np.linalg.norm(p) for p in v]
    # faces: every triple of mutually adjacent vertices (edge length 2 before
    # normalisation), oriented outward
    P = np.array(verts)
    n = len(P)
    d2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    edge = d2.min(where=d2 > 1e-12, initial=10.0)
    adj = np.abs(d2 - edge) < 1e-9
    faces = []
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    a, b, c = P[i], P[j], P[k]
                    if np.dot(np.cross(b - a, c - a), a + b + c) > 0:
                        faces.append((i, j, k))
                    else:
                        faces.append((i, k, j))
    assert len(faces) == 20
    verts = [p for p in P]
    for _ in range(subdivisions):
        cache: dict = {}
        new_faces = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    V = np.array(verts, dtype=np.float64) * radius + np.asarray(centre, dtype=np.float64)
    T = np.array(faces, dtype=np.int32)
    return Mesh(V, T, "icosphere", {"radius": radius, "centre": tuple(centre)})


# ----------------------------------------------------------------------------
# lat-long star meshes with spherical-harmonic noise
# ----------------------------------------------------------------------------

def _real_sh(l: int, m: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonic Y_lm(theta, phi), theta from +z."""
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                     * math.factorial(l - am) / math.factorial(l + am))
    p = lpmv(am, l, np.cos(theta))
    if m == 0:
        return norm * p
    if m > 0:
        return math.sqrt(2.0) * norm * p * np.cos(am * phi)
    return math.sqrt(2.0) * norm * p * np.sin(am * phi)


def _legendre_factor(l: int, m: int, theta: np.ndarray) -> np.ndarray:
    """theta factor N_l|m| P_l^|m|(cos theta) of the real harmonic."""
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                     * math.factorial(l - am) / math.factorial(l + am))
    return norm * lpmv(am, l, np.cos(theta))


def _trig(m: int, phi: np.ndarray) -> np.ndarray:
    """phi factor of the real harmonic, with the sqrt(2) of m != 0 folded in."""
    if m == 0:
        return np.ones_like(phi)
    if m > 0:
        return math.sqrt(2.0) * np.cos(m * phi)
    return math.sqrt(2.0) * np.sin(-m * phi)


def sh_coefficients(seed: int, lmax: int = 8) -> list:
    """a_lm ~ N(0, 1/l^2), drawn with NumPy PCG64 in order l = 1..lmax, m = -l..l."""
    rng = np.random.Generator(np.random.PCG64(seed))
    coeffs = []
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            coeffs.append((l, m, float(rng.normal(0.0, 1.0 / l))))
    return coeffs


def latlong_star(n_theta: int, n_phi: int, radius: float, centre, seed: int,
                 domain: int, amplitude: float = 0.25, lmax: int = 8,
                 dtype=np.float64, max_redraws: int = 50) -> Mesh:
    """Closed lat-long mesh r(theta, phi) = R (1 + A * sum a_lm Y_lm).

    Vertices: north pole, (n_theta - 1) rings of n_phi vertices, south pole.
    Each (band, sector) quad gives triangles (i,j),(i+1,j),(i+1,j+1) and
    (i,j),(i+1,j+1),(i,j+1); ring 0 / ring n_theta are the poles, so the
    2*n_phi pole-adjacent triangles that repeat a pole vertex have zero area.
    The radial graph over the sphere is star-shaped w.r.t. the centre.
    A draw is rejected (seed += 1000) if any vertex has r < R/4 or lies
    outside [4, domain - 4]^3.
    """
    c = np.asarray(centre, dtype=np.float64)
    theta_r = np.arange(1, n_theta) * (math.pi / n_theta)
    phi_r = np.arange(n_phi) * (2.0 * math.pi / n_phi)
    TH, PH = np.meshgrid(theta_r, phi_r, indexing="ij")
    th = np.concatenate([[0.0], TH.ravel(), [math.pi]])
    ph = np.concatenate([[0.0], PH.ravel(), [0.0]])
    used_seed = seed
    for _ in range(max_redraws):
        coeffs = sh_coefficients(used_seed, lmax)
        # the sum is separable on the lat-long grid: Legendre factors per ring
        # times trigonometric factors per sector (poles evaluated directly)
        ring = np.zeros((n_theta - 1, n_phi))
        poles = np.zeros(2)
        for (l, m, a) in coeffs:
            ring += a * np.outer(_legendre_factor(l, m, theta_r), _trig(m, phi_r))
            poles += a * _real_sh(l, m, np.array([0.0, math.pi]), np.zeros(2))
        s = np.concatenate([[poles[0]], ring.ravel(), [poles[1]]])
        r = radius * (1.0 + amplitude * s)
        V = np.stack([r * np.sin(th) * np.cos(ph),
                      r * np.sin(th) * np.sin(ph),
                      r * np.cos(th)], axis=1) + c
        if r.min() >= 0.25 * radius and V.min() >= 4.0 and V.max() <= domain - 4.0:
            break
        used_seed += 1000
    else:
        raise RuntimeError("no admissible noise draw")
    V = V.astype(dtype)
    north, south = 0, 1 + (n_theta - 1) * n_phi

    def vid(i, j):
        if i == 0:
            return np.full_like(j, north)
        if i == n_theta:
            return np.full_like(j, south)
        return 1 + (i - 1) * n_phi + (j % n_phi)

    tris = []
    j = np.arange(n_phi)
    for i in range(n_theta):
        a, b, cc, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
        t1 = np.stack([a, b, cc], axis=1)
        t2 = np.stack([a, cc, d], axis=1)
        tris.append(np.stack([t1, t2], axis=1).reshape(-1, 3))
    T = np.concatenate(tris).astype(np.int32)
    return Mesh(V, T, f"latlong{n_theta}x{n_phi}",
                {"radius": radius, "centre": tuple(centre), "seed": used_seed,
                 "n_theta": n_theta, "n_phi": n_phi})


# ----------------------------------------------------------------------------
# axis-aligned box and prism (cylinder)
# ----------------------------------------------------------------------------

def box(lo, hi) -> Mesh:
    """Axis-aligned box, 12 triangles, diagonals through the box corners."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    V = np.array([[(hi if (k >> a) & 1 else lo)[a] for a in range(3)]
                  for k in range(8)], dtype=np.float64)
    # vertex k has x = bit0, y = bit1, z = bit2
    quads = [
        (0, 4, 6, 2),  # x = lo, normal -x
        (1, 3, 7, 5),  # x = hi, normal +x
        (0, 1, 5, 4),  # y = lo, normal -y
        (2, 6, 7, 3),  # y = hi, normal +y
        (0, 2, 3, 1),  # z = lo, normal -z
        (4, 5, 7, 6),  # z = hi, normal +z
    ]
    T = []
    for (a, b, c, d) in quads:
        T.append((a, b, c))
        T.append((a, c, d))
    return Mesh(V, np.array(T, dtype=np.int32), "box", {"lo": tuple(lo), "hi": tuple(hi)})


def prism(n_seg: int = 256, axis_xy=(128.5, 128.5), radius: float = 30.0,
          z0: float = 100.5, z1: float = 160.5) -> Mesh:
    """Regular n_seg-gon prism along z (a faceted cylinder), capped by fans
    from the axis points.  Rim vertices are built in the first octant and
    reflected, so that symmetric vertices are exactly symmetric and the
    vertices at multiples of 90 degrees sit exactly on (axis +/- r)."""
    assert n_seg % 8 == 0
    cx, cy = axis_xy
    q = n_seg // 8
    ang = [2.0 * math.pi * k / n_seg for k in range(q + 1)]
    first = [(radius * math.cos(a), radius * math.sin(a)) for a in ang]
    first[0] = (radius, 0.0)
    # exact symmetry about the 45-degree line for the last point
    s = radius * math.sqrt(0.5)
    first[q] = (s, s)
    pts = [None] * n_seg
    for k in range(q + 1):
        x, y = first[k]
        pts[k] = (x, y)                       # 0..45
        pts[2 * q - k] = (y, x)               # 45..90
    for k in range(2 * q + 1):
        x, y = pts[k]
        pts[4 * q - k] = (-x, y)              # 90..180
    for k in range(4 * q + 1, n_seg):
        x, y = pts[n_seg - k]
        pts[k] = (x, -y)                      # 180..360
    pts[2 * q] = (0.0, radius)
    pts[4 * q] = (-radius, 0.0)
    pts[6 * q] = (0.0, -radius)
    rim = np.array(pts, dtype=np.float64) + np.array([cx, cy])
    V = np.zeros((2 * n_seg + 2, 3), dtype=np.float64)
    V[:n_seg, :2] = rim
    V[:n_seg, 2] = z0
    V[n_seg:2 * n_seg, :2] = rim
    V[n_seg:2 * n_seg, 2] = z1
    bot, top = 2 * n_seg, 2 * n_seg + 1
    V[bot] = (cx, cy, z0)
    V[top] = (cx, cy, z1)
    T = []
    for k in range(n_seg):
        k1 = (k + 1) % n_seg
        a, b = k, k1                 # bottom ring
        c, d = n_seg + k1, n_seg + k  # top ring
        T.append((a, b, c))
        T.append((a, c, d))
        T.append((bot, b, a))        # bottom cap, normal -z
        T.append((top, n_seg + k, n_seg + k1))  # top cap, normal +z
    return Mesh(V, np.array(T, dtype=np.int32), f"prism{n_seg}",
                {"axis": (cx, cy), "radius": radius, "z": (z0, z1)})


def merge(meshes, name="scene") -> Mesh:
    vs, ts, off = [], [], 0
    for m in meshes:
        vs.append(m.verts.astype(np.float64))
        ts.append(m.tris.astype(np.int64) + off)
        off += m.nv
    return Mesh(np.concatenate(vs), np.concatenate(ts).astype(np.int32), name)


def sphere_scene(n_theta=80, n_phi=100, radius=8.0, domain=256, grid=4,
                 pos_seed=5, noise_seed0=100, jitter=16.0) -> Mesh:
    """grid^3 disjoint noisy lat-long spheres at 64(i+1/2) + U(-16,16)^3."""
    rng = np.random.Generator(np.random.PCG64(pos_seed))
    spacing = domain / grid
    parts = []
    k = 0
    for iz in range(grid):
        for iy in range(grid):
            for ix in range(grid):
                base = np.array([ix, iy, iz], dtype=np.float64) * spacing + spacing / 2
                c = base + rng.uniform(-jitter, jitter, size=3)
                parts.append(latlong_star(n_theta, n_phi, radius, c, noise_seed0 + k, domain))
                k += 1
    return merge(parts, f"spheres{grid**3}x{2*n_theta*n_phi}")


# ----------------------------------------------------------------------------
# mesh checks (input contract): closed, edge-manifold, oriented, positive volume
# ----------------------------------------------------------------------------

def nondegenerate_mask(m: Mesh) -> np.ndarray:
    V = m.verts.astype(np.float64)
    T = m.tris
    n = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    return np.abs(n).sum(1) > 0


def check_closed_oriented(m: Mesh) -> None:
    """Every directed edge of a non-degenerate triangle is matched by exactly
    one opposite directed edge (closed, consistently oriented, edge-manifold)."""
    T = m.tris[nondegenerate_mask(m)].astype(np.int64)
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    nv = m.nv
    key = e[:, 0] * nv + e[:, 1]
    rkey = e[:, 1] * nv + e[:, 0]
    uk, cnt = np.unique(key, return_counts=True)
    if cnt.max() != 1:
        raise ValueError("repeated directed edge")
    if not np.all(np.isin(rkey, uk)):
        raise ValueError("open or inconsistently oriented edge")


def signed_volume(m: Mesh) -> float:
    V = m.verts.astype(np.float64)
    T = m.tris
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)
