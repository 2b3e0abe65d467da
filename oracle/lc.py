"""Long-characteristics brute force (test infrastructure only).

The exact column density along the straight ray from the centre of the
source cell to the centre of cell p, obtained by cutting the ray at every
cell face it crosses and summing n_HI * (segment length) * alpha over the
segments (Section 3: the long-characteristics method, O(N) work per cell).
Short characteristics approximate this; the two are compared with a bound,
not for equality.
"""
from __future__ import annotations

import numpy as np


def column_to_centre(nHI: np.ndarray, alpha: float, src, d) -> float:
    """Column (cm^-2) from the source centre to the centre of the cell at
    offset d (periodic grid, d inside the periodic extent)."""
    N = nHI.shape[0]
    d = np.asarray(d, dtype=np.float64)
    L = float(np.sqrt((d * d).sum()))
    if L == 0.0:
        return 0.0
    ts = [0.0, 1.0]
    for a in range(3):
        if d[a] != 0:
            n = int(abs(d[a]))
            k = np.arange(n) + 0.5                     # faces at +-0.5, +-1.5, ...
            ts.extend((k / abs(d[a])).tolist())
    ts = np.unique(np.clip(np.array(ts), 0.0, 1.0))
    mid = 0.5 * (ts[1:] + ts[:-1])
    seg = (ts[1:] - ts[:-1]) * L
    cells = np.rint(mid[:, None] * d[None, :]).astype(np.int64) + np.asarray(src)[None, :]
    cells %= N
    return float(alpha * np.sum(nHI[cells[:, 0], cells[:, 1], cells[:, 2]] * seg))
