"""Helpers for the GPU parity tests (inputs, comparisons, light-cone crops)."""
from __future__ import annotations

import numpy as np


def inner(a, r):
    return a[tuple(slice(r, s - r) for s in a.shape)]


def maxrel(got, want) -> float:
    """max |got - want| / |want| over all elements; a nonzero value where
    want == 0 counts as infinite error."""
    g = np.asarray(got, dtype=np.float64)
    w = np.asarray(want, dtype=np.float64)
    den = np.abs(w)
    bad = (den == 0) & (g != 0)
    if np.any(bad):
        return float("inf")
    den = np.where(den == 0, 1.0, den)
    return float(np.max(np.abs(g - w) / den)) if g.size else 0.0


def crop_box(n, lo, hi, r, margin):
    """Padded-coordinate slices of a crop that covers interior [lo, hi) per
    axis (x, y, z order in n/lo/hi) plus `margin` interior cells and an
    r-wide halo; the crop is clipped at the real halo.  Returns (slices in
    array order z, y, x; offset of the compared region inside the crop)."""
    sl, off = [], []
    for a in range(len(n)):
        a0 = max(lo[a] - margin, 0)
        a1 = min(hi[a] + margin, n[a])
        sl.append(slice(a0, a1 + 2 * r))  # padded coordinates: interior a0 -> a0 + r
        off.append((lo[a] - a0, hi[a] - a0))
    return tuple(reversed(sl)), tuple(reversed(off))


def compare_region(crop_result, off, r):
    """Region of a cropped oracle result that matches [lo, hi)."""
    return crop_result[tuple(slice(o0 + r, o1 + r) for o0, o1 in off)]
