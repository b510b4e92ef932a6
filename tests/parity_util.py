"""Comparison measures shared by the GPU parity tests.

nrel:     normwise relative error ||a - b||_F / ||b||_F.
elem_rel: the largest entrywise error relative to the entry itself, with a floor of
          1e-3 of the largest entry: max_i |a_i - b_i| / (|b_i| + 1e-3 max_j |b_j|).  A
          single entry that is 1% off fails it even where the normwise error of a large
          array stays small.
"""
import numpy as np


def nrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


def elem_rel(a, b, floor=1e-3):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    den = np.abs(b) + floor * max(float(np.abs(b).max()), 1e-300)
    return float((np.abs(a - b) / den).max())


def rel(a, b):
    """Relative difference of two scalars."""
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)


def comp_rel(a, b, mag):
    """Componentwise error of a product against the magnitude of its terms:
    max_i |a_i - b_i| / mag_i, where mag = |M| |X| (the product of the absolute values) is
    the scale that bounds the rounding of each entry; entries with mag_i = 0 must match
    exactly."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mag = np.asarray(mag, dtype=np.float64)
    d = np.abs(a - b)
    zero = mag == 0
    if np.any(d[zero] != 0):
        return float("inf")
    return float((d[~zero] / mag[~zero]).max()) if np.any(~zero) else 0.0
