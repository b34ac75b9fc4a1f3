"""Pins of the oracle's exact predicates against Python's exact rationals.

A Fraction holds any double exactly, so the determinant evaluated with
Fractions is the exact value.  Inputs mix random points with constructed
degenerate ones (collinear / coplanar points on dyadic grids, and one-ulp
nudges of them), where a plain floating-point evaluation is unreliable.
"""
from fractions import Fraction as F

import numpy as np
import pytest


def sgn(x):
    return (x > 0) - (x < 0)


def o2_ref(a, b, c):
    ax, ay, bx, by, cx, cy = map(F, (a[0], a[1], b[0], b[1], c[0], c[1]))
    return sgn((ax - cx) * (by - cy) - (ay - cy) * (bx - cx))


def o3_ref(a, b, c, d):
    A = [[F(float(p[k])) - F(float(d[k])) for k in range(3)] for p in (a, b, c)]
    det = (A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
           - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
           + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]))
    return sgn(det)


def _cases2(rng, n):
    out = []
    for _ in range(n):
        kind = rng.integers(4)
        a, b = rng.uniform(0, 200, 2), rng.uniform(0, 200, 2)
        if kind == 0:
            c = rng.uniform(0, 200, 2)
        elif kind == 1:  # on the line through a, b at a dyadic parameter
            a, b = np.round(a * 64) / 64, np.round(b * 64) / 64
            s = rng.integers(-8, 9) / 8.0
            c = a + s * (b - a)
        elif kind == 2:  # one-ulp nudge off the line
            a, b = np.round(a * 64) / 64, np.round(b * 64) / 64
            c = a + 0.5 * (b - a)
            c[rng.integers(2)] = np.nextafter(c[0], np.inf) if rng.integers(2) else np.nextafter(c[1], -np.inf)
        else:  # nearly collinear, random doubles
            t = rng.uniform()
            c = a + t * (b - a)
        out.append((a, b, c))
    return out


def _cases3(rng, n):
    out = []
    for _ in range(n):
        kind = rng.integers(4)
        a, b, c = (rng.uniform(0, 200, 3) for _ in range(3))
        if kind == 0:
            d = rng.uniform(0, 200, 3)
        elif kind == 1:  # coplanar at dyadic barycentrics
            a, b, c = (np.round(p * 32) / 32 for p in (a, b, c))
            u, v = rng.integers(-8, 9, 2) / 8.0
            d = a + u * (b - a) + v * (c - a)
        elif kind == 2:  # one-ulp nudge off the plane
            a, b, c = (np.round(p * 32) / 32 for p in (a, b, c))
            d = a + 0.25 * (b - a) + 0.5 * (c - a)
            k = rng.integers(3)
            d[k] = np.nextafter(d[k], np.inf if rng.integers(2) else -np.inf)
        else:  # nearly coplanar random doubles
            u, v = rng.uniform(size=2)
            d = a + u * (b - a) + v * (c - a)
        out.append((a, b, c, d))
    return out


def test_orient2d_matches_fractions(oracle_lib):
    rng = np.random.default_rng(7)
    for (a, b, c) in _cases2(rng, 3000):
        ref = o2_ref(a, b, c)
        assert oracle_lib.orient2d(a, b, c) == ref
        assert oracle_lib.lib().or_orient2d_exact(*map(float, (*a, *b, *c))) == ref


def test_orient3d_matches_fractions(oracle_lib):
    rng = np.random.default_rng(8)
    zero = 0
    for (a, b, c, d) in _cases3(rng, 3000):
        ref = o3_ref(a, b, c, d)
        zero += ref == 0
        assert oracle_lib.orient3d(a, b, c, d) == ref
        assert oracle_lib.orient3d(a, b, c, d, exact_only=True) == ref
    assert zero > 300  # the degenerate constructions really are degenerate


def test_orient3d_sign_convention(oracle_lib):
    # n = (b-a) x (c-a) = +z for the CCW unit triangle; a point below (-z) is positive
    a, b, c = (0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)
    assert oracle_lib.orient3d(a, b, c, (0.2, 0.2, -1.0)) == 1
    assert oracle_lib.orient3d(a, b, c, (0.2, 0.2, 1.0)) == -1
    assert oracle_lib.orient2d((0, 0), (1, 0), (0, 1)) == 1


def test_hit_parameter_exact_on_dyadic_case(oracle_lib):
    """A link crossing a triangle: t is a dyadic rational, returned exactly,
    both from the orient3d values and by the oracle's nearest-hit search."""
    import ctypes as C
    from synth.meshes import Mesh
    L = oracle_lib.lib()
    a = np.array([0.0, -1.0, 0.375]); b = np.array([0.0, 1.0, 0.375]); c = np.array([1.0, 0.0, 0.375])
    X = np.array([0.25, 0.0, 0.125]); Y = np.array([0.25, 0.0, 0.625])
    # exact segment/plane parameter: (0.375 - 0.125) / 0.5 = 0.5
    sx = L.or_orient3d_value(*[np.ascontiguousarray(p).ctypes.data_as(C.c_void_p) for p in (a, b, c, X)])
    sy = L.or_orient3d_value(*[np.ascontiguousarray(p).ctypes.data_as(C.c_void_p) for p in (a, b, c, Y)])
    assert sx / (sx - sy) == 0.5
    # one triangle in the plane z = 0.3125; the level-2 link from the centre
    # (0.375, 0.375, 0.125) along +z (k = 22) reaches it at t = 0.1875 / 0.25 = 0.75
    m = Mesh(np.array([[0.125, 0.125, 0.3125], [1.0, 0.125, 0.3125], [0.125, 1.0, 0.3125]]),
             np.array([[0, 1, 2]], np.int32))
    r = oracle_lib.q_points(m, (4, 4, 4), 2, np.array([[1, 1, 0]], np.int32), np.array([22], np.uint8))
    assert r["q"][0] == 0.75 and r["tri"][0] == 0 and r["tied"][0] == 0
    # the same link along -z (k = 4) misses it: no hit
    r = oracle_lib.q_points(m, (4, 4, 4), 2, np.array([[1, 1, 0]], np.int32), np.array([4], np.uint8))
    assert r["tri"][0] == -1
