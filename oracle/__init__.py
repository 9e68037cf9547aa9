"""TEST INFRASTRUCTURE ONLY: the checking implementation of sector tracking.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It wraps ``tpc_oracle.cpp`` (plain C++, built with g++ by
``build()``), which shares no code with the GPU library.

Entry points:
    track(cs, params, precision=32)   neighbour finder, cleaning, start hits,
                                      tracklet constructor (Section 2 of the paper)
    replay(cs, params, tracklets)     FP64 re-run of given attachment decisions
    propagate / update                single steps, for the closed-form pins
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tpc_oracle.cpp")
SOURCES = [SRC, os.path.join(HERE, "tpc_refit.cpp"), os.path.join(HERE, "tpc_select.cpp"),
           os.path.join(HERE, "tpc_fit.cpp"), os.path.join(HERE, "tpc_rebuild.cpp"),
           os.path.join(HERE, "tpc_merge.cpp")]
HEADERS = [os.path.join(HERE, "kalman.h")]
LIB = os.path.join(HERE, "libtpc_oracle.so")

CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-shared", "-fPIC"]


def build(extra_flags=(), out=LIB):
    """Compile the oracle with g++ (strict IEEE, no FMA contraction)."""
    cmd = ["g++", *CXXFLAGS, *extra_flags, *SOURCES, "-o", out]
    subprocess.run(cmd, check=True)
    return out


class OrcParams(ctypes.Structure):
    _fields_ = [("win_y", ctypes.c_float), ("win_z", ctypes.c_float), ("d2_max", ctypes.c_float),
                ("chi2_max", ctypes.c_float), ("sinphi_max", ctypes.c_float),
                ("u_max", ctypes.c_float), ("sigma_y", ctypes.c_float),
                ("sigma_z", ctypes.c_float), ("cww0", ctypes.c_float), ("bz", ctypes.c_float),
                ("min_hits", ctypes.c_int32), ("max_misses", ctypes.c_int32),
                ("descent_rows", ctypes.c_int32), ("brute", ctypes.c_int32)]


@dataclass
class Params:
    """Tracking parameters (readings of the paper; values in cm, GeV/c, T)."""
    win_y: float = 2.0
    win_z: float = 2.0
    d2_max: float = 0.36
    chi2_max: float = 16.0
    sinphi_max: float = 0.99
    u_max: float = 0.1
    sigma_y: float = 0.1
    sigma_z: float = 0.1
    cww0: float = 100.0
    bz: float = 0.5
    min_hits: int = 10
    max_misses: int = 8
    descent_rows: int = 8

    def c_struct(self, brute=False):
        return OrcParams(self.win_y, self.win_z, self.d2_max, self.chi2_max, self.sinphi_max,
                         self.u_max, self.sigma_y, self.sigma_z, self.cww0, self.bz,
                         self.min_hits, self.max_misses, self.descent_rows, 1 if brute else 0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
                os.path.getmtime(f) for f in SOURCES + HEADERS):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.orc_track.restype = P
        L.orc_track.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, P, P,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_free.argtypes = [P]
        L.orc_nf_margins.restype = ctypes.c_int64
        L.orc_nf_margins.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P, P, P, ctypes.c_double, P]
        L.orc_margins.restype = ctypes.c_int64
        L.orc_margins.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P, P, P, ctypes.c_double,
                                  ctypes.c_double, P]
        L.orc_len.restype = ctypes.c_int64
        L.orc_len.argtypes = [P, ctypes.c_char_p]
        L.orc_get.restype = ctypes.c_int
        L.orc_get.argtypes = [P, ctypes.c_char_p, P]
        L.orc_replay.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, P, ctypes.c_int64, P, P, P,
                                 P, P, P, P, P, P, P, P]
        L.orc_propagate.restype = ctypes.c_int
        L.orc_propagate.argtypes = [ctypes.c_int, P, P, ctypes.c_double]
        L.orc_update.restype = ctypes.c_double
        L.orc_update.argtypes = [ctypes.c_int, P, P, ctypes.c_double, ctypes.c_double]
        L.orc_map_ncoef.restype = ctypes.c_int
        L.orc_map_eval.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.orc_map_correct.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, P]
        L.orc_map_basis.restype = ctypes.c_int
        L.orc_map_basis.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P]
        L.orc_refit.argtypes = [P, P, ctypes.c_int64] + [P] * 9 + [ctypes.c_int32, ctypes.c_double, P, P]
        L.orc_refit_grad.argtypes = [P, P, ctypes.c_int64] + [P] * 12
        L.orc_fit.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, ctypes.c_int64] + [P] * 14
        L.orc_rebuild.argtypes = [ctypes.c_int, P, ctypes.c_int, P] + [ctypes.c_float] * 5 + [
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_int32, ctypes.c_int64] + [P] * 17
        L.orc_merge_views.restype = ctypes.c_int
        L.orc_merge_views.argtypes = [P, P, ctypes.c_int, ctypes.c_int64, P, P, P, P]
        L.orc_merge.restype = ctypes.c_int
        L.orc_merge.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32] + [P] * 9
        L.orc_select.restype = ctypes.c_int64
        L.orc_select.argtypes = [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_int32, P, P]
        _lib = L
    return _lib


_DTYPES = {
    "link_up": np.int32, "link_down": np.int32, "clean_up": np.int32, "clean_down": np.int32,
    "starts": np.int64, "t_start": np.int64, "t_hit_begin": np.int64, "t_unit": np.int32,
    "t_r0": np.int32, "t_n": np.int32, "t_flags": np.int32, "t_row_ref": np.int32,
    "t_ndf": np.int32, "t_hits": np.int32, "t_rows": np.uint8, "t_param": np.float64,
    "t_cov": np.float64, "t_chi2": np.float64, "t_xref": np.float64, "counters": np.int64,
}


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def track(cs, params: Params | None = None, precision=32, brute=False, units=None,
          n_threads=0, row_x=None):
    """Run the whole sector tracking on a ClusterSet; returns a dict of arrays.

    Tracklet arrays (prefix ``t_``) hold one entry per start hit, kept or not;
    ``kept`` marks those with at least ``min_hits`` clusters.
    """
    from synth import geometry as G
    params = params or Params()
    xr = np.ascontiguousarray(row_x if row_x is not None else G.row_x(), dtype=np.float32)
    rb = np.ascontiguousarray(cs.row_begin, dtype=np.int64)
    y = np.ascontiguousarray(cs.y, dtype=np.float32)
    z = np.ascontiguousarray(cs.z, dtype=np.float32)
    ps = params.c_struct(brute)
    lo, hi = (-1, -1) if units is None else units
    L = lib()
    h = L.orc_track(precision, _p(xr), len(xr), ctypes.byref(ps), cs.n_units, _p(rb), _p(y),
                    _p(z), lo, hi, n_threads)
    try:
        out = {}
        for name, dt in _DTYPES.items():
            n = L.orc_len(h, name.encode())
            a = np.empty(n, dtype=dt)
            L.orc_get(h, name.encode(), _p(a))
            out[name] = a
    finally:
        L.orc_free(h)
    out["t_param"] = out["t_param"].reshape(-1, 5)
    out["t_cov"] = out["t_cov"].reshape(-1, 15)
    out["kept"] = out["t_n"] >= params.min_hits
    c = out.pop("counters")
    out["counters"] = dict(nf_pairs=int(c[0]), propagations=int(c[1]), searches=int(c[2]),
                           window_candidates=int(c[3]), attached=int(c[4]), chain=int(c[5]),
                           box_candidates=int(c[6]))
    return out


def nf_margins(cs, eps=1e-5, params: Params | None = None, row_x=None, constructor=False,
               eps_gap=1e-3):
    """Clusters whose neighbour-finder decision lies within eps (relative,
    at least absolute) of a threshold when evaluated in double: a window
    test, the D cut, or the gap between the best and second-best D; with
    constructor=True also the chi2 cut and the propagation guards (within eps)
    and the best-vs-second chi2 gap (within eps_gap) of every search of the
    double-precision constructor.  Returns a bool array over the clusters."""
    from synth import geometry as G
    params = params or Params()
    xr = np.ascontiguousarray(row_x if row_x is not None else G.row_x(), dtype=np.float32)
    rb = np.ascontiguousarray(cs.row_begin, dtype=np.int64)
    y = np.ascontiguousarray(cs.y, dtype=np.float32)
    z = np.ascontiguousarray(cs.z, dtype=np.float32)
    flags = np.zeros(len(y), np.uint8)
    ps = params.c_struct()
    if constructor:
        lib().orc_margins(_p(xr), len(xr), ctypes.byref(ps), cs.n_units, _p(rb), _p(y), _p(z),
                          float(eps), float(eps_gap), _p(flags))
    else:
        lib().orc_nf_margins(_p(xr), len(xr), ctypes.byref(ps), cs.n_units, _p(rb), _p(y), _p(z),
                             float(eps), _p(flags))
    return flags.astype(bool)


def kept_tracklets(res):
    """Compact the kept tracklets of a track() result into the output layout."""
    k = np.nonzero(res["kept"])[0]
    hb = res["t_hit_begin"]
    n = res["t_n"][k].astype(np.int64)
    hit_begin = np.zeros(len(k) + 1, dtype=np.int64)
    np.cumsum(n, out=hit_begin[1:])
    hits = np.concatenate([res["t_hits"][hb[i]:hb[i + 1]] for i in k]) if len(k) else np.zeros(0, np.int32)
    rows = np.concatenate([res["t_rows"][hb[i]:hb[i + 1]] for i in k]) if len(k) else np.zeros(0, np.uint8)
    return dict(index=k, unit=res["t_unit"][k], n=res["t_n"][k], r0=res["t_r0"][k],
                flags=res["t_flags"][k], start=res["t_start"][k], hit_begin=hit_begin,
                hits=hits, rows=rows, param=res["t_param"][k], cov=res["t_cov"][k],
                chi2=res["t_chi2"][k], xref=res["t_xref"][k], ndf=res["t_ndf"][k],
                row_ref=res["t_row_ref"][k])


def replay(cs, tk, params: Params | None = None, precision=64, row_x=None):
    """Re-run the constructor arithmetic with the given decisions forced.

    ``tk`` is a dict as returned by kept_tracklets (hit_begin, hits, rows, r0,
    flags).  Returns param [n,5], cov [n,15], chi2, xref, ok flags and smax,
    the largest |sin(phi)| the replayed trajectory reaches.
    """
    from synth import geometry as G
    params = params or Params()
    xr = np.ascontiguousarray(row_x if row_x is not None else G.row_x(), dtype=np.float32)
    y = np.ascontiguousarray(cs.y, dtype=np.float32)
    z = np.ascontiguousarray(cs.z, dtype=np.float32)
    n = len(tk["r0"])
    hb = np.ascontiguousarray(tk["hit_begin"], dtype=np.int64)
    hits = np.ascontiguousarray(tk["hits"], dtype=np.int32)
    rows = np.ascontiguousarray(tk["rows"], dtype=np.uint8)
    r0 = np.ascontiguousarray(tk["r0"], dtype=np.int32)
    fl = np.ascontiguousarray(tk["flags"], dtype=np.int32)
    param = np.zeros((n, 5))
    cov = np.zeros((n, 15))
    chi2 = np.zeros(n)
    xref = np.zeros(n)
    ok = np.zeros(n, dtype=np.int32)
    smax = np.zeros(n)
    ps = params.c_struct()
    lib().orc_replay(precision, _p(xr), len(xr), ctypes.byref(ps), _p(y), _p(z), n, _p(hb),
                     _p(hits), _p(rows), _p(r0), _p(fl), _p(param), _p(cov), _p(chi2), _p(xref),
                     _p(ok), _p(smax))
    return dict(param=param, cov=cov, chi2=chi2, xref=xref, ok=ok.astype(bool), smax=smax)


STATE_FIELDS = ("x", "y", "z", "s", "t", "w", "cyy", "csy", "css", "cwy", "cws", "cww",
                "czz", "ctz", "ctt")


def propagate(state, x1, params: Params | None = None, precision=64):
    """One propagation step; state is a length-15 vector (see STATE_FIELDS)."""
    params = params or Params()
    st = np.ascontiguousarray(state, dtype=np.float64).copy()
    ps = params.c_struct()
    ok = lib().orc_propagate(precision, ctypes.byref(ps), _p(st), float(x1))
    return st, bool(ok)


def update(state, my, mz, params: Params | None = None, precision=64):
    """One Kalman update; returns (new state, chi2)."""
    params = params or Params()
    st = np.ascontiguousarray(state, dtype=np.float64).copy()
    ps = params.c_struct()
    ch = lib().orc_update(precision, ctypes.byref(ps), _p(st), float(my), float(mz))
    return st, ch


# ---------------------------------------------------------------------------
# refit through the distortion-correction map
# ---------------------------------------------------------------------------
def map_ncoef():
    return int(lib().orc_map_ncoef())


def map_eval(theta, r, phi, z):
    """(delta r, delta r*phi, delta z) of the map at one point."""
    out = np.zeros(3)
    th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
    lib().orc_map_eval(_p(th) if th is not None else None, float(r), float(phi), float(z), _p(out))
    return out


def map_correct(theta, x, y, z, alpha):
    """Corrected (x, y, z) of a cluster measured at (x, y, z) in the frame of a
    sector centred at azimuth alpha, as the refit corrects it."""
    th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_map_correct(_p(th) if th is not None else None, float(x), float(y), float(z),
                          float(alpha), _p(out))
    return out


def map_basis(r, phi, z):
    """Non-zero basis terms at a point: (node indices [n,3] (phi, r, z), weights [n])."""
    idx = np.zeros(3 * 64, np.int32)
    w = np.zeros(64)
    n = lib().orc_map_basis(float(r), float(phi), float(z), _p(idx), _p(w))
    return idx[:3 * n].reshape(n, 3), w[:n]


def _refit_args(cs, tk, params, row_x, unit_alpha):
    from synth import geometry as G
    params = params or Params()
    xr = np.ascontiguousarray(row_x if row_x is not None else G.row_x(), dtype=np.float32)
    hb = np.ascontiguousarray(tk["hit_begin"], dtype=np.int64)
    hits = np.ascontiguousarray(tk["hits"], dtype=np.int32)
    rows = np.ascontiguousarray(tk["rows"], dtype=np.uint8)
    unit = np.ascontiguousarray(tk["unit"], dtype=np.int32)
    if unit_alpha is None:
        unit_alpha = G.sector_alpha(cs.unit_sector)
    ua = np.ascontiguousarray(unit_alpha, dtype=np.float32)
    seed = np.ascontiguousarray(tk["param"], dtype=np.float32)
    y = np.ascontiguousarray(cs.y, dtype=np.float32)
    z = np.ascontiguousarray(cs.z, dtype=np.float32)
    keep = [xr, hb, hits, rows, unit, ua, seed, y, z]
    return params.c_struct(), keep


def refit(cs, tk, theta=None, params: Params | None = None, row_x=None, unit_alpha=None, map_z=None):
    """FP64 refit chi2 of every track in tk (hit lists sorted by row; seeds from
    tk["param"]).  map_z: evaluate the map at this z for every cluster (time
    frames) instead of the measured z.  Returns (chi2 [n], ok [n])."""
    ps, (xr, hb, hits, rows, unit, ua, seed, y, z) = _refit_args(cs, tk, params, row_x, unit_alpha)
    n = len(hb) - 1
    th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
    chi2 = np.zeros(n)
    ok = np.zeros(n, np.int32)
    lib().orc_refit(_p(xr), ctypes.byref(ps), n, _p(hb), _p(hits), _p(rows), _p(unit), _p(ua),
                    _p(seed), _p(y), _p(z), _p(th) if th is not None else None,
                    0 if map_z is None else 1, 0.0 if map_z is None else float(map_z), _p(chi2), _p(ok))
    return chi2, ok.astype(bool)


def refit_grad(cs, tk, theta=None, dL_dchi2=None, params: Params | None = None, row_x=None,
               unit_alpha=None, hit_grad=False):
    """FP64 gradient of sum(dL_dchi2 * chi2) with respect to the map
    coefficients (and, optionally, to every corrected cluster coordinate)."""
    ps, (xr, hb, hits, rows, unit, ua, seed, y, z) = _refit_args(cs, tk, params, row_x, unit_alpha)
    n = len(hb) - 1
    th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
    w = np.ones(n) if dL_dchi2 is None else np.ascontiguousarray(dL_dchi2, dtype=np.float64)
    g = np.zeros(map_ncoef())
    hgrad = np.zeros((int(hb[-1]), 3)) if hit_grad else None
    lib().orc_refit_grad(_p(xr), ctypes.byref(ps), n, _p(hb), _p(hits), _p(rows), _p(unit), _p(ua),
                         _p(seed), _p(y), _p(z), _p(th) if th is not None else None, _p(w), _p(g),
                         _p(hgrad) if hit_grad else None)
    return (g, hgrad) if hit_grad else g


def select_tracks(tk, min_hits=20, index=None):
    """Sub-list of tracklets (kept_tracklets layout) with at least min_hits
    clusters, optionally restricted to the given positions."""
    sel = np.nonzero(tk["n"] >= min_hits)[0]
    if index is not None:
        sel = sel[np.asarray(index)]
    hb = tk["hit_begin"]
    n = tk["n"][sel].astype(np.int64)
    nb = np.zeros(len(sel) + 1, np.int64)
    np.cumsum(n, out=nb[1:])
    hits = np.concatenate([tk["hits"][hb[i]:hb[i + 1]] for i in sel]) if len(sel) else np.zeros(0, np.int32)
    rows = np.concatenate([tk["rows"][hb[i]:hb[i + 1]] for i in sel]) if len(sel) else np.zeros(0, np.uint8)
    return dict(index=sel, unit=tk["unit"][sel], n=tk["n"][sel], hit_begin=nb, hits=hits, rows=rows,
                param=tk["param"][sel])


def select(tk, n_clusters, shared=(1, 10)):
    """Ambiguity solving of kept tracklets (kept_tracklets layout: unit, n,
    hit_begin, hits sorted by row, chi2, ndf): returns (keep [n_tracklets]
    bool, assign [n_clusters] int32: the selected tracklet each cluster is
    assigned to, or -1).  shared = (num, den): the allowed fraction of shared
    clusters, counted from the outermost row."""
    n_tr = len(tk["n"])
    unit = np.ascontiguousarray(tk["unit"], dtype=np.int32)
    n = np.ascontiguousarray(tk["n"], dtype=np.int32)
    hb = np.ascontiguousarray(tk["hit_begin"], dtype=np.int64)
    hits = np.ascontiguousarray(tk["hits"], dtype=np.int32)
    chi2 = np.ascontiguousarray(tk["chi2"], dtype=np.float32)
    ndf = np.ascontiguousarray(tk["ndf"], dtype=np.int32)
    keep = np.zeros(n_tr, np.uint8)
    assign = np.zeros(n_clusters, np.int32)
    lib().orc_select(n_tr, _p(unit), _p(n), _p(hb), _p(hits), _p(chi2), _p(ndf), int(n_clusters),
                     int(shared[0]), int(shared[1]), _p(keep), _p(assign))
    return keep.astype(bool), assign


FIT_DEFAULTS = dict(chi2_cut=16.0, vs=1e-2, vt=1e-2, vw=1.0)


def fit(cs, tk, precision=32, reject=None, params: Params | None = None, row_x=None, **fit_params):
    """Three-iteration fit with interpolation-based cluster rejection of the
    tracks in tk (kept_tracklets layout: hit_begin, hits, rows, param, xref).
    precision 32 takes the rejection decisions; pass ``reject`` (uint8 per
    hit) with precision 64 to replay given decisions in FP64.  Returns a dict:
    param [n,5], cov [n,15], chi2, x_out, n_kept, ok, reject [hits]."""
    from synth import geometry as G
    params = params or Params()
    fp = dict(FIT_DEFAULTS, **fit_params)
    xr = np.ascontiguousarray(row_x if row_x is not None else G.row_x(), dtype=np.float32)
    hb = np.ascontiguousarray(tk["hit_begin"], dtype=np.int64)
    hits = np.ascontiguousarray(tk["hits"], dtype=np.int32)
    rows = np.ascontiguousarray(tk["rows"], dtype=np.uint8)
    seed = np.ascontiguousarray(tk["param"], dtype=np.float32)
    xref = np.ascontiguousarray(tk["xref"], dtype=np.float32)
    y = np.ascontiguousarray(cs.y, dtype=np.float32)
    z = np.ascontiguousarray(cs.z, dtype=np.float32)
    n = len(hb) - 1
    decide = reject is None
    rej = np.zeros(len(hits), np.uint8) if decide else np.ascontiguousarray(reject, dtype=np.uint8).copy()
    out = dict(param=np.zeros((n, 5)), cov=np.zeros((n, 15)), chi2=np.zeros(n), x_out=np.zeros(n),
               n_kept=np.zeros(n, np.int32), ok=np.zeros(n, np.int32))
    ps = params.c_struct()
    lib().orc_fit(precision, 1 if decide else 0, _p(xr), ctypes.byref(ps), fp["chi2_cut"], fp["vs"], fp["vt"],
                  fp["vw"], n, _p(hb), _p(hits), _p(rows), _p(seed), _p(xref), _p(y), _p(z), _p(rej),
                  _p(out["param"]), _p(out["cov"]), _p(out["chi2"]), _p(out["x_out"]), _p(out["n_kept"]),
                  _p(out["ok"]))
    out["ok"] = out["ok"].astype(bool)
    out["reject"] = rej
    return out


REBUILD_DEFAULTS = dict(chi2_cut=16.0, chi2_final=16.0, vs=1e-2, vt=1e-2, vw=1.0, k_max=4, rounds=6,
                        extrapolate=False, chi2_extrap=9.0)


def rebuild(cs, tk, precision=32, params: Params | None = None, row_x=None, **kw):
    """Phase II rebuild of the tracks in tk (kept_tracklets layout plus xref,
    chi2, ndf, unit) against the clusters of their units (cs.row_begin, y,
    z); with extrapolate=True also Phase III's candidates beyond the tracks'
    ends (chi2 cut chi2_extrap).  Returns param, cov, chi2, x_out, n_kept, ok and assigned [n, n_rows]
    (the cluster kept at each row, -1 for none)."""
    from synth import geometry as G
    params = params or Params()
    f = dict(REBUILD_DEFAULTS, **kw)
    xr = np.ascontiguousarray(row_x if row_x is not None else G.row_x(), dtype=np.float32)
    R = len(xr)
    n = len(tk["hit_begin"]) - 1
    arrs = dict(unit=np.ascontiguousarray(tk["unit"], dtype=np.int32),
                hb=np.ascontiguousarray(tk["hit_begin"], dtype=np.int64),
                hits=np.ascontiguousarray(tk["hits"], dtype=np.int32),
                rows=np.ascontiguousarray(tk["rows"], dtype=np.uint8),
                seed=np.ascontiguousarray(tk["param"], dtype=np.float32),
                xref=np.ascontiguousarray(tk["xref"], dtype=np.float32),
                chi2=np.ascontiguousarray(tk["chi2"], dtype=np.float32),
                ndf=np.ascontiguousarray(tk["ndf"], dtype=np.int32),
                rb=np.ascontiguousarray(cs.row_begin, dtype=np.int64),
                y=np.ascontiguousarray(cs.y, dtype=np.float32), z=np.ascontiguousarray(cs.z, dtype=np.float32))
    out = dict(assigned=np.zeros((n, R), np.int32), param=np.zeros((n, 5)), cov=np.zeros((n, 15)),
               chi2=np.zeros(n), x_out=np.zeros(n), n_kept=np.zeros(n, np.int32), ok=np.zeros(n, np.int32))
    ps = params.c_struct()
    a = arrs
    lib().orc_rebuild(precision, _p(xr), R, ctypes.byref(ps), f["chi2_cut"], f["chi2_final"], f["vs"], f["vt"],
                      f["vw"], int(f["k_max"]), int(f["rounds"]), int(bool(f["extrapolate"])), f["chi2_extrap"],
                      int(cs.n_units), n, _p(a["unit"]), _p(a["hb"]),
                      _p(a["hits"]), _p(a["rows"]), _p(a["seed"]), _p(a["xref"]), _p(a["chi2"]), _p(a["ndf"]),
                      _p(a["rb"]), _p(a["y"]), _p(a["z"]), _p(out["assigned"]), _p(out["param"]), _p(out["cov"]),
                      _p(out["chi2"]), _p(out["x_out"]), _p(out["n_kept"]), _p(out["ok"]))
    out["ok"] = out["ok"].astype(bool)
    return out


class OrcMergeParams(ctypes.Structure):
    _fields_ = [("x_m", ctypes.c_float), ("cos_h", ctypes.c_float), ("sin_h", ctypes.c_float),
                ("tol", ctypes.c_float * 5), ("chi2_cut", ctypes.c_float), ("cross_electrode", ctypes.c_int32)]


# merging: views at the plane between the pad rows, tolerances of (y, z,
# sin phi, dz/ds, q/pT) and the chi2 cut (readings; the paper gives none)
MERGE_DEFAULTS = dict(x_m=165.0, tol=(1.0, 1.0, 0.02, 0.02, 0.1), chi2_cut=25.0, cross_electrode=True)


def merge_params(**kw):
    """The merging parameters as the C struct; cos/sin of half the sector
    opening are rounded once from double."""
    import math
    from synth import geometry as G
    f = dict(MERGE_DEFAULTS, **kw)
    return OrcMergeParams(float(f["x_m"]), math.cos(G.HALF_OPENING_RAD), math.sin(G.HALF_OPENING_RAD),
                          (ctypes.c_float * 5)(*f["tol"]), float(f["chi2_cut"]), int(bool(f["cross_electrode"])))


def unit_neighbours(unit_sector, unit_group=None):
    """[n_units, 3]: the unit of the next sector of the same half, of the
    previous one, and of the same azimuth across the central electrode, in the
    same group (time-frame slice), -1 where there is none."""
    from synth import geometry as G
    sec = np.asarray(unit_sector, dtype=np.int64)
    grp = np.zeros(len(sec), np.int64) if unit_group is None else np.asarray(unit_group, dtype=np.int64)
    S = G.SECTORS_PER_SIDE
    where = {(int(g), int(s)): u for u, (g, s) in enumerate(zip(grp, sec))}
    nbr = -np.ones((len(sec), 3), np.int32)
    for u, (g, s) in enumerate(zip(grp, sec)):
        side, loc = divmod(int(s), S)
        for k, other in enumerate((side * S + (loc + 1) % S, side * S + (loc - 1) % S, (1 - side) * S + loc)):
            nbr[u, k] = where.get((int(g), other), -1)
    return nbr


def merge_views(tk, precision=64, params: Params | None = None, **kw):
    """Views [n, 3, 5] and their flags [n, 3] of the tracks in tk (param at
    xref, in their sector frames)."""
    params = params or Params()
    n = len(tk["param"])
    prm = np.ascontiguousarray(tk["param"], dtype=np.float32)
    xr = np.ascontiguousarray(tk["xref"], dtype=np.float32)
    views = np.zeros((n, 3, 5))
    ok = np.zeros((n, 3), np.uint8)
    ps, mp = params.c_struct(), merge_params(**kw)
    lib().orc_merge_views(ctypes.byref(ps), ctypes.byref(mp), precision, n, _p(prm), _p(xr), _p(views), _p(ok))
    return views, ok.astype(bool)


def merge(tk, unit_nbr, n_units, params: Params | None = None, **kw):
    """Track merging (FP32 decisions) of the tracks in tk (unit order; param
    at xref; r_in, r_out).  Returns prev, next, root."""
    params = params or Params()
    n = len(tk["param"])
    a = dict(unit=np.ascontiguousarray(tk["unit"], dtype=np.int32),
             prm=np.ascontiguousarray(tk["param"], dtype=np.float32),
             xr=np.ascontiguousarray(tk["xref"], dtype=np.float32),
             r_in=np.ascontiguousarray(tk["r_in"], dtype=np.int32),
             r_out=np.ascontiguousarray(tk["r_out"], dtype=np.int32),
             nbr=np.ascontiguousarray(unit_nbr, dtype=np.int32))
    out = {k: np.zeros(n, np.int32) for k in ("prev", "next", "root")}
    ps, mp = params.c_struct(), merge_params(**kw)
    lib().orc_merge(ctypes.byref(ps), ctypes.byref(mp), n, int(n_units), _p(a["unit"]), _p(a["prm"]), _p(a["xr"]),
                    _p(a["r_in"]), _p(a["r_out"]), _p(a["nbr"]), _p(out["prev"]), _p(out["next"]), _p(out["root"]))
    return out
