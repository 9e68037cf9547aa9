"""Tolerances of float results against the FP64 replay of the same decisions.

Parameters: |dp| <= 1e-4 * max(|p|, unit) + 1e-3 * sigma_p, with units
(10 cm, 10 cm, 1, 1, 1 (GeV/c)^-1) for (y, z, sin phi, dz/ds, q/pT).  The first
term is "1e-4 relative"; the second covers parameters the clusters barely
constrain (the curvature of short tracklets), whose float rounding scales with
their own standard deviation.
Covariance: |dC_ij| <= 1e-2 * max(|C_ij|, sqrt(C_ii C_jj)) (the standard-form
update cancels digits in float).  chi2: |dchi2| <= 1e-3 * max(chi2, 1).
"""
import numpy as np

UNIT = np.array([10.0, 10.0, 1.0, 1.0, 1.0])
II = [0, 1, 1, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 4]
JJ = [0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4]


def sigma(cov15):
    return np.sqrt(np.maximum(cov15[:, [0, 2, 5, 9, 14]], 0.0))


def param_bad(p, ref_p, ref_cov):
    tol = 1e-4 * np.maximum(np.abs(ref_p), UNIT) + 1e-3 * sigma(ref_cov)
    return np.abs(p - ref_p) > tol


def cov_bad(c, ref_cov):
    d = ref_cov[:, [0, 2, 5, 9, 14]]
    scale = np.maximum(np.abs(ref_cov), np.sqrt(d[:, II] * d[:, JJ]))
    return np.abs(c - ref_cov) > 1e-2 * scale


def chi2_bad(c, ref):
    return np.abs(c - ref) > 1e-3 * np.maximum(ref, 1.0)
