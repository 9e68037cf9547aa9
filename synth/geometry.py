"""Detector description used by the synthetic inputs.

The TPC is split into two halves of 18 trapezoidal sectors each (paper,
Section 2).  Within a sector the pad rows are planes at fixed distance x from
the beam axis, measured along the sector's centre line.  The paper gives no
row table; the workloads place 152 rows linearly between 85 cm and 245 cm.

This module holds the detector description only.  It contains none of the
tracking method's arithmetic; both the checking implementation and the GPU
library receive these values as inputs.
"""
from __future__ import annotations

import math

import numpy as np

N_ROWS = 152
ROW_X_FIRST_CM = 85.0
ROW_X_LAST_CM = 245.0
N_SECTORS = 36
SECTORS_PER_SIDE = 18
HALF_OPENING_RAD = math.radians(10.0)
BZ_TESLA = 0.5
Z_MAX_CM = 250.0
DRIFT_CM_PER_US = 2.58
OUTER_RADIUS_CM = 250.0
# transverse radius of curvature [cm] = pT[GeV/c] / (C_LIGHT_GEV * Bz[T])
C_LIGHT_GEV = 2.99792458e-3


def row_x_f64() -> np.ndarray:
    """Row-plane distances in cm, float64 (linear spacing)."""
    r = np.arange(N_ROWS, dtype=np.float64)
    return ROW_X_FIRST_CM + r * (ROW_X_LAST_CM - ROW_X_FIRST_CM) / (N_ROWS - 1)


def row_x() -> np.ndarray:
    """Row-plane distances as the float32 table handed to the trackers."""
    return row_x_f64().astype(np.float32)


def sector_alpha(sector) -> np.ndarray:
    """Azimuth of the centre line of a sector (0-17 side A, 18-35 side C)."""
    s = np.asarray(sector) % SECTORS_PER_SIDE
    return (s + 0.5) * (2.0 * math.pi / SECTORS_PER_SIDE)


def sector_side_is_a(sector) -> np.ndarray:
    return np.asarray(sector) < SECTORS_PER_SIDE


def tan_half_opening() -> float:
    return math.tan(HALF_OPENING_RAD)
