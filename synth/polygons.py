"""Seeded 2D geometries: closed polygons given as vertices [nv, 2] (float64,
base-cell units) and edges [ne, 2] (vertex index pairs, counter-clockwise
around each solid region)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Polygon:
    verts: np.ndarray   # [nv, 2] float64
    edges: np.ndarray   # [ne, 2] int32

    @property
    def ne(self) -> int:
        return int(self.edges.shape[0])

    @property
    def nv(self) -> int:
        return int(self.verts.shape[0])


def _ring(pts: np.ndarray) -> Polygon:
    n = len(pts)
    e = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).astype(np.int32)
    return Polygon(np.ascontiguousarray(pts, dtype=np.float64), e)


def union(*polys: Polygon) -> Polygon:
    """Disjoint polygons as one edge set."""
    vs, es, base = [], [], 0
    for p in polys:
        vs.append(p.verts)
        es.append(p.edges + base)
        base += p.nv
    return Polygon(np.concatenate(vs), np.concatenate(es).astype(np.int32))


def circle(n_edges: int, centre, radius: float, noise: float = 0.0, seed: int = 0) -> Polygon:
    """Regular n-gon inscribed in a circle, optionally with radial noise
    (relative amplitude noise, seeded), counter-clockwise."""
    rng = np.random.default_rng(seed)
    a = 2 * np.pi * np.arange(n_edges) / n_edges
    r = radius * (1.0 + noise * rng.uniform(-1, 1, n_edges)) if noise else np.full(n_edges, radius)
    pts = np.stack([centre[0] + r * np.cos(a), centre[1] + r * np.sin(a)], axis=1)
    return _ring(pts)


def rectangle(lo, hi) -> Polygon:
    """Axis-aligned rectangle [lo, hi], counter-clockwise."""
    return _ring(np.array([[lo[0], lo[1]], [hi[0], lo[1]], [hi[0], hi[1]], [lo[0], hi[1]]], dtype=np.float64))


def star(n_points: int, centre, r_out: float, r_in: float, phase: float = 0.1) -> Polygon:
    """Non-convex star polygon with n_points tips."""
    k = np.arange(2 * n_points)
    a = np.pi * k / n_points + phase
    r = np.where(k % 2 == 0, r_out, r_in)
    return _ring(np.stack([centre[0] + r * np.cos(a), centre[1] + r * np.sin(a)], axis=1))
