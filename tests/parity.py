"""Comparison helpers of the GPU parity tests (no test functions here).

Whole-field relative L2 dilutes an error confined to the boundary band, where
the closure rows and the SATs act (a few per cent of the points), so every
apply comparison also bounds the error on that band alone, in the max norm.
"""
import numpy as np

TOL = {'f64': 1e-11, 'f32': 1e-5}
BAND = {6: 9, 4: 6, 2: 2}    # closure rows of D2^FC plus the SAT reach: the frame width


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def band_mask(n1, n2, width):
    """Points closer than `width` to any face of an n1 x n2 block, shape (n2, n1)."""
    i = np.arange(n1)
    j = np.arange(n2)
    di = np.minimum(i, n1 - 1 - i)[None, :]
    dj = np.minimum(j, n2 - 1 - j)[:, None]
    return np.minimum(di, dj) < width


def band_max_rel(got, ref, order):
    """max |got - ref| / max |ref| over the boundary band of every block.

    got, ref: lists of (2, n2, n1) arrays (one per block) or one such array."""
    if isinstance(got, np.ndarray) and got.ndim == 3:
        got, ref = [got], [ref]
    err = scale = 0.0
    for g, r in zip(got, ref):
        g, r = np.asarray(g, dtype=float), np.asarray(r, dtype=float)
        m = band_mask(r.shape[2], r.shape[1], BAND[order])
        err = max(err, float(np.abs(g - r)[:, m].max()))
        scale = max(scale, float(np.abs(r)[:, m].max()))
    return err / scale
