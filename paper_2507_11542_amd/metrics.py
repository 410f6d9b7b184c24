"""Error measures for level-set results: zero-set extraction and Hausdorff
distance in cell units, and per-region max-abs errors.

Measurement only (numpy/scipy); nothing here is part of the solver.

Zero set of a nodal field V: every grid edge whose end values change sign
(V <= 0 against V > 0) contributes the linear-interpolation crossing point,
and every node with V == 0 contributes itself.  Points are in index units, so
distances are in cells; periodic axes wrap.
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np


def zero_set_points(v: np.ndarray, periodic: Sequence[bool]) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    nd = v.ndim
    pts = []
    idx = np.indices(v.shape, dtype=np.float64)
    for d in range(nd):
        if periodic[d]:
            a = v
            b = np.roll(v, -1, axis=d)
            sl = tuple(slice(None) for _ in range(nd))
        else:
            sl = tuple(slice(0, -1) if k == d else slice(None) for k in range(nd))
            sl_b = tuple(slice(1, None) if k == d else slice(None) for k in range(nd))
            a = v[sl]
            b = v[sl_b]
        cross = (a <= 0.0) != (b <= 0.0)
        if not np.any(cross):
            continue
        av = a[cross]
        bv = b[cross]
        frac = av / (av - bv)
        coords = np.stack([idx[k][sl][cross] for k in range(nd)], axis=1)
        coords[:, d] += frac
        if periodic[d]:
            coords[:, d] = np.mod(coords[:, d], v.shape[d])
        pts.append(coords)
    zeros = np.argwhere(v == 0.0).astype(np.float64)
    if zeros.size:
        pts.append(zeros)
    if not pts:
        return np.zeros((0, nd))
    return np.concatenate(pts, axis=0)


def hausdorff_cells(va: np.ndarray, vb: np.ndarray, periodic: Sequence[bool]) -> float:
    """Symmetric Hausdorff distance (in cells) between the zero sets of va, vb."""
    from scipy.spatial import cKDTree

    pa = zero_set_points(va, periodic)
    pb = zero_set_points(vb, periodic)
    if len(pa) == 0 and len(pb) == 0:
        return 0.0
    if len(pa) == 0 or len(pb) == 0:
        return float("inf")
    box = np.array([float(s) if p else 10.0 * s + 10.0
                    for s, p in zip(va.shape, periodic)])
    pa = np.mod(pa, box)
    pb = np.mod(pb, box)
    ta = cKDTree(pa, boxsize=box)
    tb = cKDTree(pb, boxsize=box)
    dab, _ = tb.query(pa)
    dba, _ = ta.query(pb)
    return float(max(dab.max(), dba.max()))


def region_errors(v: np.ndarray, ref: np.ndarray, dx: Sequence[float],
                  periodic: Sequence[bool], band_cells: float = 3.0,
                  edge_cells: int = 6) -> Dict[str, float]:
    """Max-abs error overall, in the front band |ref| < band_cells*max(dx),
    in that band away from the bounded edges (band_inner), within edge_cells
    of a bounded edge, and in the rest (interior)."""
    v = np.asarray(v, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(v - ref)
    band = np.abs(ref) < band_cells * float(np.max(dx))
    edge = np.zeros(ref.shape, dtype=bool)
    for d, p in enumerate(periodic):
        if p:
            continue
        idx = np.arange(ref.shape[d])
        near = (idx < edge_cells) | (idx >= ref.shape[d] - edge_cells)
        shape = [1] * ref.ndim
        shape[d] = ref.shape[d]
        edge |= near.reshape(shape)
    interior = ~band & ~edge

    def mx(mask):
        return float(err[mask].max()) if np.any(mask) else 0.0

    return {"max_abs": float(err.max()) if err.size else 0.0, "band": mx(band),
            "band_inner": mx(band & ~edge), "edge": mx(edge), "interior": mx(interior)}
