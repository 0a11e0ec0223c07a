"""Restoration quality measures of Sec. 4.

Test infrastructure only (see the package docstring).

The paper's E(X^) is "the mean gray-level of the uncontaminated image"; it is
read as the mean over all entries of the tensor.
"""
import numpy as np


def relative_error(X_true, X):
    """||X^ - X_restored||_F / ||X^||_F."""
    X_true = np.asarray(X_true, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    return float(np.linalg.norm((X_true - X).ravel()) / np.linalg.norm(X_true.ravel()))


def snr(X_true, X):
    """10 log10(||X^ - E(X^)||_F^2 / ||X_restored - X^||_F^2)."""
    X_true = np.asarray(X_true, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    num = np.sum((X_true - X_true.mean()) ** 2)
    den = np.sum((X - X_true) ** 2)
    return float(10.0 * np.log10(num / den))
