"""Shared pieces of the patch-test pins and GPU parity tests."""
import numpy as np

from oracle import fem as ofem


def oracle_patch(pt, kappa, mortar=False):
    return ofem.patch_test(pt, kappa, mortar=mortar)


def stress_errors(pt, x):
    """(max relative sigma_zz error, max spurious stress) over all tetrahedra."""
    s = ofem.stress(pt.X, pt.tets, pt.young, pt.poisson, x)
    zz = np.abs(s[:, 2, 2] + pt.pressure) / pt.pressure
    other = np.abs(s)
    other[:, 2, 2] = 0.0
    return float(zz.max()), float(other.max())
