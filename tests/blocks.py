"""Sampled checks of full-size launches: blocks of the grid against the oracle applied to
the block alone.

A step's output at a point depends only on its inputs within the step's reach, so the
oracle's step applied to a small block of the inputs gives the full grid's value at every
point of the block whose reach stays inside the block, or crosses a side of the block that
is the grid's own boundary (where the oracle and the kernels both take the odd extension).
`tests/test_blocks.py` checks these cores against the oracle's full-grid results.
"""
import numpy as np


def core(starts, B, n, margin):
    """Per-axis slices of a B-wide block at `starts` (grid side n): the points at least
    `margin` inside the block, or nearer a block side that is the grid's boundary."""
    return tuple(slice(0 if a == 0 else margin, B if a + B == n else B - margin) for a in starts)


def starts(n, B, centres, even=False):
    """Block starts around the given centres (clipped to the grid; even for blocks that
    carry a coarse block)."""
    out = []
    for c in centres:
        a = min(max(c - B // 2, 0), n - B)
        if even:
            a -= a % 2
        out.append(a)
    return sorted(set(out))


# Block sizes and margins (in block points) of each step, radius-2 cross operator.
SWEEP_B, SWEEP_M = 9, 2           # a sweep or defect reads u within 2 of the point
RR_B, RR_CB, RR_M = 17, 9, 2      # defect + full weighting: coarse j reads fine 2j-3 .. 2j+3
PRO_B, PRO_CB, PRO_M = 17, 9, 4   # cubic interpolation: fine i reads coarse i/2-1 .. i/2+2


def cut(a, st, B):
    """The B-wide block of a (numpy array, or a device tensor read back as FP64) at st."""
    b = a[tuple(slice(s, s + B) for s in st)]
    if isinstance(b, np.ndarray):
        return np.array(b)
    return b.double().cpu().numpy()


def coarse(st):
    """Starts of the coarse block under a fine block at (even) st."""
    return [a // 2 for a in st]
