"""Seeded loss weights for the cut-link table (inputs of the gradient check).

w = 2u - 1 with u the top 53 bits of splitmix64(seed ^ key) scaled by 2^-53,
key a hash of the link's identity (level, block coordinates, cell, direction),
so that weights do not depend on the order of the table.
"""
import numpy as np

M64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def link_weights(level: int, bcoord: np.ndarray, cell: np.ndarray, dirs: np.ndarray, seed: int = 3) -> np.ndarray:
    b = cell.astype(np.int64) // 64
    t = cell.astype(np.int64) % 64
    bc = bcoord[b].astype(np.uint64)
    with np.errstate(over="ignore"):
        key = np.uint64(level)
        key = key * np.uint64(1 << 20) + bc[:, 0]
        key = key * np.uint64(1 << 20) + bc[:, 1]
        key = key * np.uint64(1 << 20) + bc[:, 2]
        key = key * np.uint64(64 * 27) + t.astype(np.uint64) * np.uint64(27) + dirs.astype(np.uint64)
    u = (splitmix64(key ^ np.uint64(seed)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return 2.0 * u - 1.0
