"""Named synthetic workloads (meshes + grid settings).

Each workload fixes the mesh, the base grid n0 (cells per axis, multiple of 4),
the finest level L_f (levels 0..L_f), the lattice (19 or 27 directions) and the
near-wall distance d_spec in base cells.  Sizes follow the paper's workloads:
112K / 7.2M triangles at 1024 / 4096 effective resolution (Tables 1 and 4).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import meshes, polygons


@dataclass
class Workload:
    name: str
    mesh: meshes.Mesh
    n0: tuple
    lf: int
    lattice: int
    d_spec: float = 2.0

    @property
    def levels(self):
        return list(range(self.lf + 1))


def icosphere64() -> Workload:
    """Icosphere r=12 (1,280 triangles, float64) in a uniform 64^3 grid, D3Q19."""
    return Workload("icosphere64", meshes.icosphere(3, 12.0, (32.3, 31.7, 32.1)),
                    (64, 64, 64), 0, 19)


def star112k() -> Workload:
    """Lat-long star 224x250 (112,000 triangles, float64), R=40, 128^3 base,
    levels 0..3 (1024 effective), D3Q19, d_spec = 2."""
    m = meshes.latlong_star(224, 250, 40.0, (64.3, 63.7, 64.1), seed=1, domain=128)
    return Workload("star112k", m, (128, 128, 128), 3, 19)


def star7m() -> Workload:
    """Lat-long star 1800x2000 (7,200,000 triangles, float32), R=40, 256^3 base,
    levels 0..4 (4096 effective), D3Q27, d_spec = 2."""
    m = meshes.latlong_star(1800, 2000, 40.0, (128.3, 127.7, 128.1), seed=2,
                            domain=256, dtype=np.float32)
    return Workload("star7m", m, (256, 256, 256), 4, 27)


def box256() -> Workload:
    """Axis-aligned box [100.5, 140.5625]^3: faces on level-0 and level-3
    cell-centre planes; 256^3 base, levels 0..3, D3Q19."""
    m = meshes.box((100.5,) * 3, (140.5625,) * 3)
    return Workload("box256", m, (256, 256, 256), 3, 19)


def prism256() -> Workload:
    """256-gon prism r=30 along z through (128.5, 128.5), z in [100.5, 160.5]."""
    return Workload("prism256", meshes.prism(256), (256, 256, 256), 3, 19)


def spheres64() -> Workload:
    """64 disjoint noisy lat-long spheres 80x100 (1,024,000 triangles)."""
    return Workload("spheres64", meshes.sphere_scene(), (256, 256, 256), 3, 19)


# ----------------------------------------------------------------------------
# reduced workloads: same constructions, sizes the CPU oracle finishes in seconds
# ----------------------------------------------------------------------------

def star_small(n_theta=28, n_phi=32, n0=32, lf=2, lattice=19, seed=11,
               dtype=np.float64) -> Workload:
    r = n0 * 40.0 / 128.0
    c = (n0 / 2 + 0.3, n0 / 2 - 0.3, n0 / 2 + 0.1)
    m = meshes.latlong_star(n_theta, n_phi, r, c, seed=seed, domain=n0, dtype=dtype)
    return Workload(f"star{2*n_theta*n_phi}_{n0}", m, (n0, n0, n0), lf, lattice)


def box_small(lf=2) -> Workload:
    """Box [20.5, 36.5625]^3 in a 64^3 base grid: faces on level-0 and level-3
    centre planes, so cell centres lie exactly on faces, edges and corners."""
    m = meshes.box((20.5,) * 3, (36.5625,) * 3)
    return Workload("box64", m, (64, 64, 64), lf, 19)


def prism_small(lf=2) -> Workload:
    m = meshes.prism(64, (32.5, 32.5), 12.0, 20.5, 44.5)
    return Workload("prism64", m, (64, 64, 64), lf, 19)


def spheres_small(lf=2) -> Workload:
    m = meshes.sphere_scene(n_theta=10, n_phi=12, radius=4.0, domain=64, grid=2,
                            jitter=4.0)
    return Workload("spheres8", m, (64, 64, 64), lf, 19)


# ----------------------------------------------------------------------------
# 2D (quadtrees, D2Q9): the paper's cylinder and square cases (root grid
# 512^2, D_s = N_x / 64 base cells, the square 2 D_s wide and shifted by 0.7
# base cells along x) and reduced versions for the oracle
# ----------------------------------------------------------------------------

@dataclass
class Workload2D:
    name: str
    poly: polygons.Polygon
    n0: tuple
    lf: int
    d_spec: float = 2.0
    lattice: int = 9


def cylinder2d(lf=4, n_edges=4096) -> Workload2D:
    """Circle of diameter 8 base cells (D_s = 1/64 of the unit domain) in the
    centre of a 512^2 root grid; levels 0..lf (the paper's L_max = lf + 1)."""
    return Workload2D("cylinder2d", polygons.circle(n_edges, (256.0, 256.0), 4.0), (512, 512), lf)


def square2d(lf=4) -> Workload2D:
    """Square of side 16 base cells (2 D_s) centred in a 512^2 root grid and
    shifted by 0.7 base cells along +x."""
    return Workload2D("square2d", polygons.rectangle((248.7, 248.0), (264.7, 264.0)), (512, 512), lf)


def cylinder2d_small(lf=2) -> Workload2D:
    return Workload2D("cylinder2d_small", polygons.circle(256, (32.3, 31.7), 10.0, noise=0.05, seed=3), (64, 64), lf)


def square2d_small(lf=2) -> Workload2D:
    """Edges on level-0 centre lines (x, y = k + 1/2): centres exactly on edges
    and corners."""
    return Workload2D("square2d_small", polygons.rectangle((20.5, 24.5), (40.5, 36.5)), (64, 64), lf)


def shapes2d_small(lf=3) -> Workload2D:
    """A non-convex star, a noisy circle and a small rectangle, disjoint."""
    poly = polygons.union(polygons.star(7, (20.2, 40.3), 12.0, 5.0),
                          polygons.circle(96, (46.1, 20.4), 8.0, noise=0.1, seed=5),
                          polygons.rectangle((44.25, 44.5), (52.75, 50.125)))
    return Workload2D("shapes2d_small", poly, (64, 64), lf)


REGISTRY = {
    "icosphere64": icosphere64,
    "star112k": star112k,
    "star7m": star7m,
    "box256": box256,
    "prism256": prism256,
    "spheres64": spheres64,
    "star_small": star_small,
    "box_small": box_small,
    "prism_small": prism_small,
    "spheres_small": spheres_small,
    "cylinder2d": cylinder2d,
    "square2d": square2d,
    "cylinder2d_small": cylinder2d_small,
    "square2d_small": square2d_small,
    "shapes2d_small": shapes2d_small,
}


def get(name: str, **kw) -> Workload:
    return REGISTRY[name](**kw)
