"""Tolerances of float results against the FP64 replay of the same decisions.

Parameters: |dp| <= 1e-4 * max(|p|, unit), with units (10 cm, 10 cm, 1, 1,
1 (GeV/c)^-1) for (y, z, sin phi, dz/ds, q/pT): "1e-4 relative", with a
floor for parameters near zero.
Covariance: |dC_ij| <= 1e-4 * max(|C_ij|, sqrt(C_ii C_jj)).
chi2: |dchi2| <= 1e-3 * max(chi2, 1).
Refit chi2: the same 1e-3 * max(chi2, 1) for every refitted track.

These hold because the Kalman filter keeps its covariance factorised (U D U^T,
Bierman's update: no difference of nearly equal covariances) and the tracklet
state's y and z relative to the seed cluster (their rounding scales with the
distance travelled, not with the drift coordinate of a time frame, which
reaches thousands of cm).

One class is held to ten times these bounds for parameters and covariances:
tracklets whose trajectory reaches |sin phi| >= 0.95 (the FP64 replay's
smax), within 0.04 of the 0.99 guard.  There dy/d(sin phi) and dy/d(q/pT) of
a step grow as 1/cos^3 phi (>= 33 at cos phi <= 0.31), so the ~3e-8 absolute
rounding of sin phi in float is amplified into parameter errors up to ~2e-4
relative (measured on the CPU: 3 of 515 k time-frame tracklets above 1e-4,
all with smax >= 0.98; outside the class the largest is 2.8e-5).  The class
holds 7-13 % of the tracklets of a central event (7.4 % with 10k primaries,
12.5 % with 2k primaries, where loopers weigh more); callers count it and
assert that it stays below 20 %.
"""

NEAR_GUARD = 0.95
import numpy as np

UNIT = np.array([10.0, 10.0, 1.0, 1.0, 1.0])
II = [0, 1, 1, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 4]
JJ = [0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4]


def sigma(cov15):
    return np.sqrt(np.maximum(cov15[:, [0, 2, 5, 9, 14]], 0.0))


def _rel(smax, n):
    """Relative bound per tracklet: 1e-4, or 1e-3 in the near-guard class."""
    if smax is None:
        return np.full((n, 1), 1e-4)
    return np.where(np.asarray(smax) >= NEAR_GUARD, 1e-3, 1e-4)[:, None]


def param_bad(p, ref_p, smax=None):
    return np.abs(p - ref_p) > _rel(smax, len(p)) * np.maximum(np.abs(ref_p), UNIT)


def cov_bad(c, ref_cov, smax=None):
    d = ref_cov[:, [0, 2, 5, 9, 14]]
    scale = np.maximum(np.abs(ref_cov), np.sqrt(d[:, II] * d[:, JJ]))
    return np.abs(c - ref_cov) > _rel(smax, len(c)) * scale


def chi2_bad(c, ref):
    return np.abs(c - ref) > 1e-3 * np.maximum(ref, 1.0)


def refit_chi2_bad(c, ref):
    return np.abs(c - ref) > 1e-3 * np.maximum(ref, 1.0)
