"""Edge-case workloads shared by the GPU edge tests: empty and degenerate
geometry, bodies at the ends of the coordinate range, single solid cells."""
import numpy as np

from synth import configs, meshes, polygons


def tetra(c, r, dtype=np.float64):
    """Tetrahedron around c (outward counter-clockwise faces)."""
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64) * r + np.asarray(c)
    t = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], dtype=np.int32)
    return meshes.Mesh(v.astype(dtype), t, "tetra")


def cases3d():
    n0 = (32, 32, 32)
    empty = meshes.Mesh(np.zeros((0, 3)), np.zeros((0, 3), dtype=np.int32), "empty")
    # strictly between cell centres: no centre inside, nothing refined
    between = tetra((10.0, 10.0, 10.0), 0.2)
    # one solid centre (10.5, 10.5, 10.5) at level 0
    single = tetra((10.5, 10.5, 10.5), 0.6)
    # zero-area triangles only (three collinear points, both orientations)
    flat = meshes.Mesh(np.array([[5.0, 5.0, 5.0], [6.0, 6.0, 6.0], [7.0, 7.0, 7.0]]),
                       np.array([[0, 1, 2], [0, 2, 1]], dtype=np.int32), "flat")
    # a box from the lowest allowed coordinate to the top of the domain
    edge_box = meshes.box((0.25, 0.25, 0.25), (32.0, 9.5, 32.0))
    out = {}
    for name, m in [("empty", empty), ("between", between), ("single", single), ("flat", flat),
                    ("edge_box", edge_box)]:
        out[name] = configs.Workload(name, m, n0, 2, 27)
    return out


def cases2d():
    n0 = (32, 32)
    empty = polygons.Polygon(np.zeros((0, 2)), np.zeros((0, 2), dtype=np.int32))
    single = polygons.Polygon(np.array([[10.0, 10.0], [11.2, 10.5], [10.2, 11.1]]),
                              np.array([[0, 1], [1, 2], [2, 0]], dtype=np.int32))
    edge_rect = polygons.rectangle((0.25, 0.25), (32.0, 9.5))
    out = {}
    for name, p in [("empty2d", empty), ("single2d", single), ("edge_rect2d", edge_rect)]:
        out[name] = configs.Workload2D(name, p, n0, 2)
    return out
