"""NumPy brute-force neighbour sets for tiny inputs (test infrastructure).

States the definition directly: N(i) = { j != i : |r_i - r_j|_min-image < h_i + h_j },
i.e. r_ij < 2 h_ij with h_ij = (h_i + h_j)/2, over all N^2 pairs at once.
Independent of the C oracle's loops; used to pin its neighbour search.
"""
from __future__ import annotations

import numpy as np


def pair_displacements(pos: np.ndarray, box) -> np.ndarray:
    """r_ij = r_i - r_j under the minimum-image convention, shape (D, N, N)."""
    box = np.asarray(box, dtype=np.float64).reshape(-1, 1, 1)
    d = pos[:, :, None] - pos[:, None, :]
    return d - box * np.round(d / box)


def neighbor_sets(pos: np.ndarray, h: np.ndarray, box) -> list[np.ndarray]:
    rij = pair_displacements(pos, box)
    r = np.sqrt(np.sum(rij * rij, axis=0))
    support = h[:, None] + h[None, :]
    mask = r < support
    np.fill_diagonal(mask, False)
    return [np.nonzero(mask[i])[0] for i in range(pos.shape[1])]
