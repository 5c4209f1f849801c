"""Partition comparison for the oracle (test infrastructure only).

Normalised mutual information, arithmetic normalisation:
NMI(X, Y) = 2 I(X; Y) / (H(X) + H(Y)), natural logarithm, FP64, from the
contingency table of the two labelings.  The paper names NMI as a quality
measure (Section 1) without defining it; this is the common definition of
Danon et al. (J. Stat. Mech. 2005) with arithmetic-mean normalisation.
Two single-cluster partitions give 1 by convention.
"""
import numpy as np


def _entropy(counts, n):
    p = counts[counts > 0].astype(np.float64) / n
    return float(-(p * np.log(p)).sum())


def nmi(x, y) -> float:
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    if x.shape != y.shape:
        raise ValueError("labelings differ in length")
    n = x.size
    if n == 0:
        return 1.0
    _, xi = np.unique(x, return_inverse=True)
    _, yi = np.unique(y, return_inverse=True)
    cx = np.bincount(xi)
    cy = np.bincount(yi)
    hx, hy = _entropy(cx, n), _entropy(cy, n)
    if hx + hy == 0.0:
        return 1.0
    pair = xi * (int(yi.max()) + 1) + yi
    _, cxy = np.unique(pair, return_counts=True)
    # I = sum_xy p_xy log(p_xy / (p_x p_y))
    _, first = np.unique(pair, return_index=True)
    px = cx[xi[first]].astype(np.float64) / n
    py = cy[yi[first]].astype(np.float64) / n
    pxy = cxy.astype(np.float64) / n
    mi = float((pxy * np.log(pxy / (px * py))).sum())
    return 2.0 * mi / (hx + hy)
