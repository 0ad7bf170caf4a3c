"""Map between the oracle's compact interior-edge numbering and the library's padded
edge layout (offset d B + (k (n+1) + j) P + i)."""
import numpy as np

from oracle import mesh


def padded_index(n, P, B):
    d, p = mesh.edge_coords(n)
    return d * B + (p[:, 2] * (n + 1) + p[:, 1]) * P + p[:, 0]


def to_padded(n, P, B, v):
    v = np.asarray(v)
    out = np.zeros(v.shape[:-1] + (3 * B,))
    out[..., padded_index(n, P, B)] = v
    return out


def from_padded(n, P, B, v):
    return np.asarray(v)[..., padded_index(n, P, B)]


def boundary_mask(n, P, B):
    m = np.ones(3 * B, dtype=bool)
    m[padded_index(n, P, B)] = False
    return m
