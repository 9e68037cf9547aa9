"""MI355X-native per-sector TPC track finding (arXiv 2601.20569, Section 2).

A thin ctypes binding of ``libtpcx.so`` (the C interface in include/tpcx.h).
PyTorch provides device memory and the stream; every step of the tracking
runs in the library's HIP kernels.  There is no CPU fallback: without the
built library on a gfx950 device the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

from .build import LIB

TPCX_OK = 0
TPCX_E_ARG = -1
TPCX_E_CAPACITY = -2
TPCX_E_HIP = -3
TPCX_E_DEVICE = -4
TPCX_E_INPUT = -5
ST_START_OVERFLOW, ST_TRACK_OVERFLOW, ST_HIT_OVERFLOW = 1, 2, 4


class TpcxError(RuntimeError):
    pass


class Geometry(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("row_x_host", ctypes.POINTER(ctypes.c_float)),
                ("tan_half_opening", ctypes.c_float), ("bz_tesla", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("win_y", ctypes.c_float), ("win_z", ctypes.c_float), ("d2_max", ctypes.c_float),
                ("chi2_max", ctypes.c_float), ("sinphi_max", ctypes.c_float),
                ("u_max", ctypes.c_float), ("sigma_y", ctypes.c_float),
                ("sigma_z", ctypes.c_float), ("cww0", ctypes.c_float),
                ("min_hits", ctypes.c_int32), ("max_misses", ctypes.c_int32),
                ("descent_rows", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("bin_y", ctypes.c_float), ("n_zbins", ctypes.c_int32), ("block", ctypes.c_int32),
                ("construct_grid", ctypes.c_int32), ("construct_refill", ctypes.c_int32),
                ("refit_grid", ctypes.c_int32), ("refit_refill", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Clusters(ctypes.Structure):
    _fields_ = [("n_units", ctypes.c_int32), ("n_clusters", ctypes.c_int64),
                ("row_begin", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p)]


class Tracks(ctypes.Structure):
    _fields_ = [("cap_tracks", ctypes.c_int64), ("cap_hits", ctypes.c_int64),
                ("counts", ctypes.c_void_p), ("unit", ctypes.c_void_p), ("start", ctypes.c_void_p),
                ("n_hits", ctypes.c_void_p), ("hit_begin", ctypes.c_void_p),
                ("hit_id", ctypes.c_void_p), ("hit_row", ctypes.c_void_p),
                ("x_ref", ctypes.c_void_p), ("param", ctypes.c_void_p), ("cov", ctypes.c_void_p),
                ("chi2", ctypes.c_void_p), ("ndf", ctypes.c_void_p)]


class RefitInput(ctypes.Structure):
    _fields_ = [("n_tracks", ctypes.c_int64), ("n_hits", ctypes.c_int64), ("hit_begin", ctypes.c_void_p),
                ("hit_id", ctypes.c_void_p), ("hit_row", ctypes.c_void_p),
                ("unit", ctypes.c_void_p), ("seed", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("unit_alpha", ctypes.c_void_p)]


MAP_NCOEF = 36720


class FitParams(ctypes.Structure):
    _fields_ = [("chi2_cut", ctypes.c_float), ("var_s", ctypes.c_float), ("var_t", ctypes.c_float),
                ("var_w", ctypes.c_float)]


class FitInput(ctypes.Structure):
    _fields_ = [("n_tracks", ctypes.c_int64), ("n_hits", ctypes.c_int64), ("hit_begin", ctypes.c_void_p),
                ("hit_id", ctypes.c_void_p), ("hit_row", ctypes.c_void_p), ("seed", ctypes.c_void_p),
                ("x_ref", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("n_clusters", ctypes.c_int64)]


class FitOutput(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("cov", ctypes.c_void_p), ("chi2", ctypes.c_void_p),
                ("x_out", ctypes.c_void_p), ("n_kept", ctypes.c_void_p), ("ok", ctypes.c_void_p),
                ("reject", ctypes.c_void_p)]


class RebuildParams(ctypes.Structure):
    _fields_ = [("chi2_cut", ctypes.c_float), ("chi2_final", ctypes.c_float), ("var_s", ctypes.c_float),
                ("var_t", ctypes.c_float), ("var_w", ctypes.c_float), ("rounds", ctypes.c_int32),
                ("extrapolate", ctypes.c_int32), ("chi2_extrap", ctypes.c_float)]


class RebuildInput(ctypes.Structure):
    _fields_ = [("n_tracks", ctypes.c_int64), ("n_hits", ctypes.c_int64), ("unit", ctypes.c_void_p),
                ("hit_begin", ctypes.c_void_p), ("hit_id", ctypes.c_void_p), ("hit_row", ctypes.c_void_p),
                ("seed", ctypes.c_void_p), ("x_ref", ctypes.c_void_p), ("chi2", ctypes.c_void_p),
                ("ndf", ctypes.c_void_p)]


class RebuildOutput(ctypes.Structure):
    _fields_ = [("assigned", ctypes.c_void_p), ("param", ctypes.c_void_p), ("cov", ctypes.c_void_p),
                ("chi2", ctypes.c_void_p), ("x_out", ctypes.c_void_p), ("n_kept", ctypes.c_void_p),
                ("ok", ctypes.c_void_p)]


class MergeParams(ctypes.Structure):
    _fields_ = [("x_m", ctypes.c_float), ("cos_h", ctypes.c_float), ("sin_h", ctypes.c_float),
                ("tol", ctypes.c_float * 5), ("chi2_cut", ctypes.c_float), ("cross_electrode", ctypes.c_int32)]


class MergeInput(ctypes.Structure):
    _fields_ = [("n_tracks", ctypes.c_int64), ("n_units", ctypes.c_int32), ("unit", ctypes.c_void_p),
                ("param", ctypes.c_void_p), ("x_ref", ctypes.c_void_p), ("r_in", ctypes.c_void_p),
                ("r_out", ctypes.c_void_p), ("unit_nbr", ctypes.c_void_p)]


class MergeOutput(ctypes.Structure):
    _fields_ = [("prev", ctypes.c_void_p), ("next", ctypes.c_void_p), ("root", ctypes.c_void_p)]


class BatchRefit(ctypes.Structure):
    _fields_ = [("min_hits", ctypes.c_int32), ("map_z_fixed", ctypes.c_int32), ("map_z", ctypes.c_float),
                ("theta", ctypes.c_void_p),
                ("unit_alpha", ctypes.c_void_p), ("chi2", ctypes.c_void_p), ("ok", ctypes.c_void_p)]


class Debug(ctypes.Structure):
    _fields_ = [("link_up", ctypes.c_void_p), ("link_down", ctypes.c_void_p),
                ("clean_up", ctypes.c_void_p), ("clean_down", ctypes.c_void_p),
                ("starts", ctypes.c_void_p)]


STAGES = ("grid", "neighbours", "starts", "construct", "compact", "refit")

_lib = None


def lib():
    """Load libtpcx.so (built by paper_2601_20569_amd.build.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise TpcxError(f"{LIB} is missing: build it with paper_2601_20569_amd.build.build()")
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.tpcx_default_tuning.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(Tuning)]
        L.tpcx_default_tuning.restype = None
        L.tpcx_create.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(Params),
                                  ctypes.POINTER(Tuning), ctypes.POINTER(P)]
        L.tpcx_create.restype = ctypes.c_int32
        L.tpcx_destroy.argtypes = [P]
        L.tpcx_destroy.restype = None
        L.tpcx_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64]
        L.tpcx_workspace_bytes.restype = ctypes.c_size_t
        L.tpcx_track.argtypes = [P, ctypes.POINTER(Clusters), P, ctypes.c_size_t, ctypes.c_int64,
                                 ctypes.POINTER(Tracks), ctypes.POINTER(Debug), P]
        L.tpcx_track.restype = ctypes.c_int32
        L.tpcx_track_static.argtypes = [P, ctypes.POINTER(Clusters), ctypes.c_int64,
                                        ctypes.POINTER(Tracks), ctypes.POINTER(Debug), P]
        L.tpcx_track_static.restype = ctypes.c_int32
        L.tpcx_poll.argtypes = [P, ctypes.POINTER(Tracks), P]
        L.tpcx_poll.restype = ctypes.c_int32
        L.tpcx_strerror.argtypes = [ctypes.c_int32]
        L.tpcx_strerror.restype = ctypes.c_char_p
        L.tpcx_refit_workspace_bytes.argtypes = [P, ctypes.c_int64, ctypes.c_int64]
        L.tpcx_refit_workspace_bytes.restype = ctypes.c_size_t
        L.tpcx_refit.argtypes = [P, ctypes.POINTER(RefitInput), P, P, P, P, ctypes.c_size_t, P]
        L.tpcx_refit.restype = ctypes.c_int32
        L.tpcx_refit_backward.argtypes = [P, ctypes.POINTER(RefitInput), P, P, P, ctypes.c_size_t, P]
        L.tpcx_refit_backward.restype = ctypes.c_int32
        L.tpcx_batched_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                                   ctypes.c_int64, ctypes.c_int64]
        L.tpcx_batched_workspace_bytes.restype = ctypes.c_size_t
        L.tpcx_track_batched.argtypes = [P, ctypes.POINTER(Clusters), P, ctypes.c_size_t,
                                         ctypes.c_int64, ctypes.POINTER(Tracks),
                                         ctypes.POINTER(BatchRefit), P]
        L.tpcx_track_batched.restype = ctypes.c_int32
        L.tpcx_fit_workspace_bytes.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.tpcx_fit_workspace_bytes.restype = ctypes.c_size_t
        L.tpcx_fit.argtypes = [P, ctypes.POINTER(FitInput), ctypes.POINTER(FitParams),
                               ctypes.POINTER(FitOutput), P, ctypes.c_size_t, P]
        L.tpcx_fit.restype = ctypes.c_int32
        L.tpcx_rebuild_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64]
        L.tpcx_rebuild_workspace_bytes.restype = ctypes.c_size_t
        L.tpcx_rebuild.argtypes = [P, ctypes.POINTER(Clusters), ctypes.POINTER(RebuildInput),
                                   ctypes.POINTER(RebuildParams), ctypes.POINTER(RebuildOutput), P,
                                   ctypes.c_size_t, P]
        L.tpcx_rebuild.restype = ctypes.c_int32
        L.tpcx_merge_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_int64]
        L.tpcx_merge_workspace_bytes.restype = ctypes.c_size_t
        L.tpcx_merge.argtypes = [P, ctypes.POINTER(MergeInput), ctypes.POINTER(MergeParams),
                                 ctypes.POINTER(MergeOutput), P, ctypes.c_size_t, P]
        L.tpcx_merge.restype = ctypes.c_int32
        L.tpcx_select_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_int64]
        L.tpcx_select_workspace_bytes.restype = ctypes.c_size_t
        L.tpcx_select.argtypes = [P, ctypes.POINTER(Tracks), ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_int32, P, P, P, P, ctypes.c_size_t, P]
        L.tpcx_select.restype = ctypes.c_int32
        L.tpcx_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.tpcx_set_tuning.restype = ctypes.c_int32
        L.tpcx_autotune_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                                    ctypes.c_int64, ctypes.c_int64]
        L.tpcx_autotune_workspace_bytes.restype = ctypes.c_size_t
        L.tpcx_autotune_batched.argtypes = [P, ctypes.POINTER(Clusters), P, ctypes.c_size_t, ctypes.c_int64,
                                            ctypes.POINTER(Tracks), ctypes.POINTER(BatchRefit), ctypes.c_int32,
                                            ctypes.POINTER(Tuning), P]
        L.tpcx_autotune_batched.restype = ctypes.c_int32
        L.tpcx_timing_enable.argtypes = [P, ctypes.c_int32]
        L.tpcx_timing_enable.restype = ctypes.c_int32
        L.tpcx_timing_read.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32)]
        L.tpcx_timing_read.restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(st, what):
    if st != TPCX_OK:
        raise TpcxError(f"{what}: {lib().tpcx_strerror(st).decode()} ({st})")


def unit_neighbours(unit_sector, unit_group=None, sectors_per_side=18):
    """[n_units, 3] int32 (numpy): for every unit, the unit of the next
    sector of the same half, of the previous one, and of the same azimuth
    across the central electrode, within the same group (time-frame slice);
    -1 where there is none.  Sectors 0 .. S-1 are one half, S .. 2S-1 the
    other, in the same azimuthal order."""
    import numpy as np
    sec = [int(s) for s in unit_sector]
    grp = [0] * len(sec) if unit_group is None else [int(g) for g in unit_group]
    S = int(sectors_per_side)
    index = {(g, s): u for u, (g, s) in enumerate(zip(grp, sec))}
    nbr = np.full((len(sec), 3), -1, np.int32)
    for u, (g, s) in enumerate(zip(grp, sec)):
        half, k = divmod(s, S)
        nbr[u] = [index.get((g, half * S + (k + 1) % S), -1), index.get((g, half * S + (k - 1) % S), -1),
                  index.get((g, (1 - half) * S + k), -1)]
    return nbr


def default_tuning(n_units, n_clusters):
    t = Tuning()
    lib().tpcx_default_tuning(n_units, n_clusters, ctypes.byref(t))
    return t


@dataclass
class MethodParams:
    """Values of the method's cuts (cm, GeV/c)."""
    win_y: float = 2.0
    win_z: float = 2.0
    d2_max: float = 0.36
    chi2_max: float = 16.0
    sinphi_max: float = 0.99
    u_max: float = 0.1
    sigma_y: float = 0.1
    sigma_z: float = 0.1
    cww0: float = 100.0
    min_hits: int = 10
    max_misses: int = 8
    descent_rows: int = 8

    def c_struct(self):
        return Params(self.win_y, self.win_z, self.d2_max, self.chi2_max, self.sinphi_max,
                      self.u_max, self.sigma_y, self.sigma_z, self.cww0, self.min_hits,
                      self.max_misses, self.descent_rows)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


class SectorTracker:
    """A tpcx context: geometry and parameters fixed, many calls.

    ``row_x``: pad-row plane distances (cm); ``tan_half_opening``: tan of the
    sector half-angle; ``bz``: field in T.  ``tuning`` (a Tuning) fixes the
    search grid and launch shapes; None chooses them per call.
    """

    def __init__(self, row_x, tan_half_opening, bz, params: MethodParams | None = None,
                 tuning: Tuning | None = None):
        import numpy as np
        import torch
        if not torch.cuda.is_available():
            raise TpcxError("no HIP device visible")
        self.params = params or MethodParams()
        self.row_x = np.ascontiguousarray(row_x, dtype=np.float32)
        self.n_rows = len(self.row_x)
        self.tan_half = float(tan_half_opening)
        g = Geometry(self.n_rows, self.row_x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                     float(tan_half_opening), float(bz))
        p = self.params.c_struct()
        h = ctypes.c_void_p()
        _check(lib().tpcx_create(ctypes.byref(g), ctypes.byref(p),
                                 ctypes.byref(tuning) if tuning is not None else None,
                                 ctypes.byref(h)), "tpcx_create")
        self._h = h
        self.device = torch.cuda.current_device()
        self._ws = None

    def close(self):
        if getattr(self, "_h", None):
            lib().tpcx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timing_enable(self, max_calls):
        """Record per-stage HIP events for the next max_calls track calls."""
        _check(lib().tpcx_timing_enable(self._h, int(max_calls)), "tpcx_timing_enable")

    def timing_read(self):
        """(summed ms per stage as a dict, number of recorded calls)."""
        ms = (ctypes.c_float * len(STAGES))()
        n = ctypes.c_int32()
        _check(lib().tpcx_timing_read(self._h, ms, ctypes.byref(n)), "tpcx_timing_read")
        return dict(zip(STAGES, list(ms))), int(n.value)

    def workspace_bytes(self, n_units, n_clusters, cap_start):
        return int(lib().tpcx_workspace_bytes(self._h, n_units, n_clusters, cap_start))

    def allocate(self, n_units, n_clusters, cap_start=None, cap_tracks=None, cap_hits=None,
                 workspace=True):
        """Device buffers for one call shape (workspace and outputs)."""
        import torch
        dev = torch.device("cuda", self.device)
        cap_start = int(n_clusters // 3 + 1) if cap_start is None else int(cap_start)
        cap_tracks = cap_start if cap_tracks is None else int(cap_tracks)
        cap_hits = int(max(1024, 4 * n_clusters)) if cap_hits is None else int(cap_hits)
        nb = self.workspace_bytes(n_units, n_clusters, cap_start)
        ws, off = None, 0
        if workspace:
            ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
            off = (-ws.data_ptr()) % 256
        i32, i64, f32 = torch.int32, torch.int64, torch.float32
        out = dict(
            counts=torch.zeros(4, dtype=i64, device=dev),
            unit=torch.empty(cap_tracks, dtype=i32, device=dev),
            start=torch.empty(cap_tracks, dtype=i32, device=dev),
            n_hits=torch.empty(cap_tracks, dtype=i32, device=dev),
            hit_begin=torch.empty(cap_tracks, dtype=i64, device=dev),
            hit_id=torch.empty(cap_hits, dtype=i32, device=dev),
            hit_row=torch.empty(cap_hits, dtype=torch.uint8, device=dev),
            x_ref=torch.empty(cap_tracks, dtype=f32, device=dev),
            param=torch.empty((cap_tracks, 5), dtype=f32, device=dev),
            cov=torch.empty((cap_tracks, 15), dtype=f32, device=dev),
            chi2=torch.empty(cap_tracks, dtype=f32, device=dev),
            ndf=torch.empty(cap_tracks, dtype=i32, device=dev),
        )
        return dict(ws=ws, ws_off=off, ws_bytes=nb, cap_start=cap_start, cap_tracks=cap_tracks,
                    cap_hits=cap_hits, out=out)

    def track_into(self, row_begin, y, z, n_units, bufs, debug=None, stream=None, static=False):
        """Enqueue one tpcx_track call into preallocated buffers (no sync).
        ``static``: tpcx_track_static, on the library's per-device scratch
        array instead of bufs' workspace (bufs["ws"] may then be None)."""
        import torch
        n = int(y.numel())
        for t, dt in ((row_begin, torch.int64), (y, torch.float32), (z, torch.float32)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise TpcxError("inputs must be contiguous device tensors: row_begin int64, y/z float32")
        if row_begin.numel() != n_units * self.n_rows + 1 or z.numel() != n:
            raise TpcxError("row_begin must have n_units*n_rows+1 entries and y, z the same length")
        cl = Clusters(n_units, n, _ptr(row_begin), _ptr(y), _ptr(z))
        o = bufs["out"]
        tr = Tracks(bufs["cap_tracks"], bufs["cap_hits"], _ptr(o["counts"]), _ptr(o["unit"]),
                    _ptr(o["start"]), _ptr(o["n_hits"]), _ptr(o["hit_begin"]), _ptr(o["hit_id"]),
                    _ptr(o["hit_row"]), _ptr(o["x_ref"]), _ptr(o["param"]), _ptr(o["cov"]),
                    _ptr(o["chi2"]), _ptr(o["ndf"]))
        dbg = None
        if debug is not None:
            dbg = Debug(*[_ptr(debug.get(k)) for k in ("link_up", "link_down", "clean_up",
                                                        "clean_down", "starts")])
        s = stream if stream is not None else torch.cuda.current_stream()
        if static:
            st = lib().tpcx_track_static(self._h, ctypes.byref(cl), bufs["cap_start"], ctypes.byref(tr),
                                         ctypes.byref(dbg) if dbg is not None else None,
                                         ctypes.c_void_p(s.cuda_stream))
            _check(st, "tpcx_track_static")
        else:
            ws = bufs["ws"]
            st = lib().tpcx_track(self._h, ctypes.byref(cl), ctypes.c_void_p(ws.data_ptr() + bufs["ws_off"]),
                                  bufs["ws_bytes"], bufs["cap_start"], ctypes.byref(tr),
                                  ctypes.byref(dbg) if dbg is not None else None,
                                  ctypes.c_void_p(s.cuda_stream))
            _check(st, "tpcx_track")
        self._last = (tr, s)
        return tr

    def fit(self, hit_begin, hit_id, hit_row, seed, x_ref, y, z, chi2_cut=16.0, var_s=1e-2, var_t=1e-2,
            var_w=1.0, stream=None):
        """Three-iteration fit with interpolation-based rejection (tpcx_fit) of
        the tracks given by device tensors (hit_begin int64 [n+1], hit_id int32,
        hit_row uint8, seed float32 [n,5], x_ref float32 [n], clusters y, z).
        Returns a dict of device tensors: param, cov, chi2, x_out, n_kept, ok,
        reject (no sync)."""
        import torch
        n = int(hit_begin.numel()) - 1
        nh = int(hit_id.numel())
        for v, dt in ((hit_begin, torch.int64), (hit_id, torch.int32), (hit_row, torch.uint8),
                      (seed, torch.float32), (x_ref, torch.float32), (y, torch.float32), (z, torch.float32)):
            if v.dtype != dt or not v.is_cuda or not v.is_contiguous():
                raise TpcxError("fit inputs must be contiguous device tensors of the documented types")
        if y.numel() != z.numel():
            raise TpcxError("fit: y and z must have one entry per cluster")
        nc = int(y.numel())
        dev = hit_begin.device
        f32, i32 = torch.float32, torch.int32
        out = dict(param=torch.zeros((max(n, 1), 5), dtype=f32, device=dev),
                   cov=torch.zeros((max(n, 1), 15), dtype=f32, device=dev),
                   chi2=torch.zeros(max(n, 1), dtype=f32, device=dev),
                   x_out=torch.zeros(max(n, 1), dtype=f32, device=dev),
                   n_kept=torch.zeros(max(n, 1), dtype=i32, device=dev),
                   ok=torch.zeros(max(n, 1), dtype=i32, device=dev),
                   reject=torch.zeros(max(nh, 1), dtype=torch.uint8, device=dev))
        nb = int(lib().tpcx_fit_workspace_bytes(self._h, n, nh, nc))
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        fi = FitInput(n, nh, _ptr(hit_begin), _ptr(hit_id), _ptr(hit_row), _ptr(seed), _ptr(x_ref), _ptr(y),
                      _ptr(z), nc)
        fo = FitOutput(*[_ptr(out[k]) for k in ("param", "cov", "chi2", "x_out", "n_kept", "ok", "reject")])
        fp = FitParams(chi2_cut, var_s, var_t, var_w)
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().tpcx_fit(self._h, ctypes.byref(fi), ctypes.byref(fp), ctypes.byref(fo),
                              ctypes.c_void_p(ws.data_ptr() + off), nb, ctypes.c_void_p(s.cuda_stream)),
               "tpcx_fit")
        out["_ws"] = ws
        res = {k: v[:n] for k, v in out.items() if k not in ("reject", "_ws")}
        res["reject"] = out["reject"][:nh]
        res["_ws"] = ws
        return res

    def rebuild(self, row_begin, y, z, n_units, unit, hit_begin, hit_id, hit_row, seed, x_ref, chi2, ndf,
                chi2_cut=16.0, chi2_final=16.0, var_s=1e-2, var_t=1e-2, var_w=1.0, rounds=6, extrapolate=False,
                chi2_extrap=9.0, stream=None):
        """Phase II rebuild (tpcx_rebuild) of the tracks given by device tensors
        against the clusters (row_begin, y, z of the tracking input); with
        extrapolate, Phase III's candidates beyond the tracks' ends too.  Returns a
        dict of device tensors: assigned [n, n_rows], param, cov, chi2, x_out,
        n_kept, ok (no sync)."""
        import torch
        n = int(hit_begin.numel()) - 1
        nh = int(hit_id.numel())
        for v, dt in ((row_begin, torch.int64), (y, torch.float32), (z, torch.float32), (unit, torch.int32),
                      (hit_begin, torch.int64), (hit_id, torch.int32), (hit_row, torch.uint8),
                      (seed, torch.float32), (x_ref, torch.float32), (chi2, torch.float32), (ndf, torch.int32)):
            if v.dtype != dt or not v.is_cuda or not v.is_contiguous():
                raise TpcxError("rebuild inputs must be contiguous device tensors of the documented types")
        dev = hit_begin.device
        f32, i32 = torch.float32, torch.int32
        m = max(n, 1)
        out = dict(assigned=torch.empty((m, self.n_rows), dtype=i32, device=dev),
                   param=torch.empty((m, 5), dtype=f32, device=dev), cov=torch.empty((m, 15), dtype=f32, device=dev),
                   chi2=torch.empty(m, dtype=f32, device=dev), x_out=torch.empty(m, dtype=f32, device=dev),
                   n_kept=torch.empty(m, dtype=i32, device=dev), ok=torch.empty(m, dtype=i32, device=dev))
        nc = int(y.numel())
        nb = int(lib().tpcx_rebuild_workspace_bytes(self._h, n_units, nc, n))
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        cl = Clusters(n_units, nc, _ptr(row_begin), _ptr(y), _ptr(z))
        ri = RebuildInput(n, nh, _ptr(unit), _ptr(hit_begin), _ptr(hit_id), _ptr(hit_row), _ptr(seed), _ptr(x_ref),
                          _ptr(chi2), _ptr(ndf))
        ro = RebuildOutput(*[_ptr(out[k]) for k in ("assigned", "param", "cov", "chi2", "x_out", "n_kept", "ok")])
        rp = RebuildParams(chi2_cut, chi2_final, var_s, var_t, var_w, rounds, int(bool(extrapolate)), chi2_extrap)
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().tpcx_rebuild(self._h, ctypes.byref(cl), ctypes.byref(ri), ctypes.byref(rp), ctypes.byref(ro),
                                  ctypes.c_void_p(ws.data_ptr() + off), nb, ctypes.c_void_p(s.cuda_stream)),
               "tpcx_rebuild")
        res = {k: v[:n] for k, v in out.items()}
        res["_ws"] = ws
        return res

    def merge(self, unit, param, x_ref, r_in, r_out, unit_nbr, n_units, x_m=165.0,
              tol=(1.0, 1.0, 0.02, 0.02, 0.1), chi2_cut=25.0, cross_electrode=True, half_opening=None,
              stream=None):
        """Track merging (tpcx_merge) of the tracks given by device tensors
        (unit ascending; param at x_ref in the sector frame; first and last
        row); unit_nbr [n_units, 3] int32 on the device; half_opening: half
        the sector opening in radians (default: from the geometry's tangent).
        Returns a dict of device tensors prev, next, root (no sync)."""
        import math

        import torch
        n = int(unit.numel())
        for v, dt in ((unit, torch.int32), (param, torch.float32), (x_ref, torch.float32), (r_in, torch.int32),
                      (r_out, torch.int32), (unit_nbr, torch.int32)):
            if v.dtype != dt or not v.is_cuda or not v.is_contiguous():
                raise TpcxError("merge inputs must be contiguous device tensors of the documented types")
        dev = unit.device
        m = max(n, 1)
        out = {k: torch.empty(m, dtype=torch.int32, device=dev) for k in ("prev", "next", "root")}
        nb = int(lib().tpcx_merge_workspace_bytes(self._h, int(n_units), n))
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        h = math.atan(self.tan_half) if half_opening is None else float(half_opening)
        mp = MergeParams(x_m, math.cos(h), math.sin(h), (ctypes.c_float * 5)(*tol), chi2_cut, int(bool(cross_electrode)))
        mi = MergeInput(n, int(n_units), _ptr(unit), _ptr(param), _ptr(x_ref), _ptr(r_in), _ptr(r_out), _ptr(unit_nbr))
        mo = MergeOutput(*[_ptr(out[k]) for k in ("prev", "next", "root")])
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().tpcx_merge(self._h, ctypes.byref(mi), ctypes.byref(mp), ctypes.byref(mo),
                                ctypes.c_void_p(ws.data_ptr() + off), nb, ctypes.c_void_p(s.cuda_stream)),
               "tpcx_merge")
        res = {k: v[:n] for k, v in out.items()}
        res["_ws"] = ws
        return res

    def allocate_select(self, n_units, n_clusters, cap_tracks):
        """Buffers of tpcx_select: keep flags, cluster assignment, counts, workspace."""
        import torch
        dev = torch.device("cuda", self.device)
        nb = int(lib().tpcx_select_workspace_bytes(self._h, n_units, n_clusters))
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        return dict(keep=torch.empty(max(cap_tracks, 1), dtype=torch.uint8, device=dev),
                    assign=torch.empty(max(n_clusters, 1), dtype=torch.int32, device=dev),
                    counts=torch.zeros(2, dtype=torch.int64, device=dev), ws=ws,
                    ws_off=(-ws.data_ptr()) % 256, ws_bytes=nb)

    def select_into(self, bufs, n_units, n_clusters, sel, shared=(1, 10), stream=None):
        """Enqueue tpcx_select on the tracklets a track_into / track_batched_into
        call wrote to bufs (no sync)."""
        import torch
        tr = self._tracks_struct(bufs)
        s = stream if stream is not None else torch.cuda.current_stream()
        st = lib().tpcx_select(self._h, ctypes.byref(tr), n_units, n_clusters, int(shared[0]), int(shared[1]),
                               _ptr(sel["keep"]), _ptr(sel["assign"]), _ptr(sel["counts"]),
                               ctypes.c_void_p(sel["ws"].data_ptr() + sel["ws_off"]), sel["ws_bytes"],
                               ctypes.c_void_p(s.cuda_stream))
        _check(st, "tpcx_select")

    def _tracks_struct(self, bufs):
        o = bufs["out"]
        return Tracks(bufs["cap_tracks"], bufs["cap_hits"], _ptr(o["counts"]), _ptr(o["unit"]),
                      _ptr(o["start"]), _ptr(o["n_hits"]), _ptr(o["hit_begin"]), _ptr(o["hit_id"]),
                      _ptr(o["hit_row"]), _ptr(o["x_ref"]), _ptr(o["param"]), _ptr(o["cov"]),
                      _ptr(o["chi2"]), _ptr(o["ndf"]))

    def allocate_batched(self, n_units, n_clusters, cap_start, cap_tracks, cap_hits, refit=True,
                         autotune=False):
        """Buffers for tpcx_track_batched: workspace (tracking + refit), outputs
        and the refit results.  ``autotune``: a workspace large enough for
        every tuning the autotuner tries."""
        import torch
        bufs = self.allocate(n_units, n_clusters, cap_start, cap_tracks, cap_hits)
        size = lib().tpcx_autotune_workspace_bytes if autotune else lib().tpcx_batched_workspace_bytes
        nb = int(size(self._h, n_units, n_clusters, bufs["cap_start"], bufs["cap_tracks"], bufs["cap_hits"]))
        dev = bufs["ws"].device
        bufs["ws"] = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        bufs["ws_off"] = (-bufs["ws"].data_ptr()) % 256
        bufs["ws_bytes"] = nb
        if refit:
            bufs["refit_chi2"] = torch.zeros(max(bufs["cap_tracks"], 1), dtype=torch.float32, device=dev)
            bufs["refit_ok"] = torch.zeros(max(bufs["cap_tracks"], 1), dtype=torch.int32, device=dev)
        return bufs

    def _batched_args(self, row_begin, y, z, n_units, bufs, unit_alpha, theta, refit_min_hits,
                      map_z=None):
        import torch
        n = int(y.numel())
        cl = Clusters(n_units, n, _ptr(row_begin), _ptr(y), _ptr(z))
        o = bufs["out"]
        tr = Tracks(bufs["cap_tracks"], bufs["cap_hits"], _ptr(o["counts"]), _ptr(o["unit"]),
                    _ptr(o["start"]), _ptr(o["n_hits"]), _ptr(o["hit_begin"]), _ptr(o["hit_id"]),
                    _ptr(o["hit_row"]), _ptr(o["x_ref"]), _ptr(o["param"]), _ptr(o["cov"]),
                    _ptr(o["chi2"]), _ptr(o["ndf"]))
        rf = None
        if unit_alpha is not None:
            if theta is not None and (theta.dtype != torch.float32 or theta.numel() != MAP_NCOEF):
                raise TpcxError("theta must be float32 with 36720 coefficients")
            rf = BatchRefit(int(refit_min_hits), 0 if map_z is None else 1,
                            0.0 if map_z is None else float(map_z),
                            _ptr(theta) if theta is not None else None,
                            _ptr(unit_alpha), _ptr(bufs["refit_chi2"]), _ptr(bufs["refit_ok"]))
            bufs["_refit_keep"] = (theta, unit_alpha)
        ws = ctypes.c_void_p(bufs["ws"].data_ptr() + bufs["ws_off"])
        return cl, tr, rf, ws

    def track_batched_into(self, row_begin, y, z, n_units, bufs, stream, unit_alpha=None,
                           theta=None, refit_min_hits=20, map_z=None):
        """Enqueue tpcx_track_batched (graph captured on the first call with
        these buffers, replayed afterwards).  ``stream`` must be a non-default
        torch stream.  With ``unit_alpha`` the tracklets with at least
        ``refit_min_hits`` clusters are refitted (results in bufs["refit_chi2"],
        bufs["refit_ok"]); ``map_z`` (cm): evaluate the map at this z for every
        cluster (time frames), else at the measured z."""
        if stream is None or stream.cuda_stream == 0:
            raise TpcxError("the batched form needs a non-default stream (graph capture)")
        cl, tr, rf, ws = self._batched_args(row_begin, y, z, n_units, bufs, unit_alpha, theta,
                                            refit_min_hits, map_z)
        st = lib().tpcx_track_batched(self._h, ctypes.byref(cl), ws, bufs["ws_bytes"], bufs["cap_start"],
                                      ctypes.byref(tr), ctypes.byref(rf) if rf is not None else None,
                                      ctypes.c_void_p(stream.cuda_stream))
        _check(st, "tpcx_track_batched")

    def autotune_batched(self, row_begin, y, z, n_units, bufs, stream, unit_alpha=None, theta=None,
                         refit_min_hits=20, reps=1, map_z=None):
        """Run tpcx_autotune_batched on this input (buffers from
        allocate_batched(..., autotune=True)); the chosen tuning stays in the
        context and is returned as a dict."""
        cl, tr, rf, ws = self._batched_args(row_begin, y, z, n_units, bufs, unit_alpha, theta,
                                            refit_min_hits, map_z)
        best = Tuning()
        st = lib().tpcx_autotune_batched(self._h, ctypes.byref(cl), ws, bufs["ws_bytes"], bufs["cap_start"],
                                         ctypes.byref(tr), ctypes.byref(rf) if rf is not None else None,
                                         int(reps), ctypes.byref(best), ctypes.c_void_p(stream.cuda_stream))
        _check(st, "tpcx_autotune_batched")
        return best.as_dict()

    def set_tuning(self, tuning):
        """Fix the context's tuning (a Tuning or a dict as autotune_batched
        returns); None returns to the size-dependent defaults."""
        t = None
        if tuning is not None:
            t = tuning if isinstance(tuning, Tuning) else Tuning(**tuning)
        _check(lib().tpcx_set_tuning(self._h, ctypes.byref(t) if t is not None else None), "tpcx_set_tuning")

    def track(self, row_begin, y, z, n_units, debug=False, cap_start=None, cap_tracks=None,
              cap_hits=None):
        """Track and return device tensors cut to the produced sizes.  When a
        capacity was too small the call is repeated with the required sizes
        (a larger start capacity can reveal more tracklets, hence 3 tries)."""
        import torch
        n = int(y.numel())
        for _attempt in range(3):
            bufs = self.allocate(n_units, n, cap_start, cap_tracks, cap_hits)
            dev = bufs["out"]["counts"].device
            dbg = None
            if debug:
                dbg = {k: torch.empty(max(n, 1), dtype=torch.int32, device=dev)
                       for k in ("link_up", "link_down", "clean_up", "clean_down")}
                dbg["starts"] = torch.empty(max(bufs["cap_start"], 1), dtype=torch.int32, device=dev)
            self.track_into(row_begin, y, z, n_units, bufs, dbg)
            counts = bufs["out"]["counts"].cpu().tolist()
            n_start, n_tr, n_hits, status = counts
            if status & 7 == 0:  # no capacity overflow (bit 8: non-finite input, reported)
                break
            cap_start = max(bufs["cap_start"], n_start)
            cap_tracks = max(bufs["cap_tracks"], n_tr)
            cap_hits = max(bufs["cap_hits"], n_hits)
        else:
            raise TpcxError(f"capacity still exceeded after resizing: counts={counts}")
        o = bufs["out"]
        res = {k: v[:n_tr] for k, v in o.items() if k not in ("counts", "hit_id", "hit_row")}
        res["hit_id"] = o["hit_id"][:n_hits]
        res["hit_row"] = o["hit_row"][:n_hits]
        res["n_start"] = n_start
        res["status"] = status
        if debug:
            for k in ("link_up", "link_down", "clean_up", "clean_down"):
                res[k] = dbg[k][:n]
            res["starts"] = dbg["starts"][:min(n_start, bufs["cap_start"])]
        return res


class RefitJob:
    """Refit of a fixed track list through the distortion-correction map.

    Tensors (device): hit_begin int64 [n+1], hit_id int32, hit_row uint8,
    unit int32 [n], seed float32 [n,5], y/z float32 (clusters), unit_alpha
    float32 [n_units].  The workspace holds the corrected clusters and the
    filter-state checkpoints between forward() and backward().
    """

    def __init__(self, tracker: "SectorTracker", hit_begin, hit_id, hit_row, unit, seed, y, z,
                 unit_alpha):
        import torch
        self.tracker = tracker
        self.t = dict(hit_begin=hit_begin, hit_id=hit_id, hit_row=hit_row, unit=unit, seed=seed,
                      y=y, z=z, unit_alpha=unit_alpha)
        for k, dt in (("hit_begin", torch.int64), ("hit_id", torch.int32), ("hit_row", torch.uint8),
                      ("unit", torch.int32), ("seed", torch.float32), ("y", torch.float32),
                      ("z", torch.float32), ("unit_alpha", torch.float32)):
            v = self.t[k]
            if v.dtype != dt or not v.is_cuda or not v.is_contiguous():
                raise TpcxError(f"refit input {k} must be a contiguous device {dt} tensor")
        self.n_tracks = int(hit_begin.numel()) - 1
        self.n_hits = int(hit_id.numel())
        self.c = RefitInput(self.n_tracks, self.n_hits, _ptr(hit_begin), _ptr(hit_id), _ptr(hit_row),
                            _ptr(unit), _ptr(seed), _ptr(y), _ptr(z), _ptr(unit_alpha))
        self.n_forward = 0  # forward() calls so far (backward works on the last one's workspace)
        nb = int(lib().tpcx_refit_workspace_bytes(tracker._h, self.n_tracks, self.n_hits))
        dev = hit_begin.device
        self.ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        self.ws_off = (-self.ws.data_ptr()) % 256
        self.ws_bytes = nb
        self.chi2 = torch.zeros(max(self.n_tracks, 1), dtype=torch.float32, device=dev)
        self.ok = torch.zeros(max(self.n_tracks, 1), dtype=torch.int32, device=dev)

    def _ws(self):
        return ctypes.c_void_p(self.ws.data_ptr() + self.ws_off)

    def forward(self, theta=None, stream=None):
        """chi2 per track (float32 [n]); ok flags in self.ok."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        th = None
        if theta is not None:
            if theta.dtype != torch.float32 or theta.numel() != MAP_NCOEF or not theta.is_cuda:
                raise TpcxError("theta must be a float32 device tensor of 36720 coefficients")
            th = theta.contiguous()
        _check(lib().tpcx_refit(self.tracker._h, ctypes.byref(self.c), _ptr(th) if th is not None else None,
                                _ptr(self.chi2), _ptr(self.ok), self._ws(), self.ws_bytes,
                                ctypes.c_void_p(s.cuda_stream)), "tpcx_refit")
        self.n_forward += 1
        return self.chi2[:self.n_tracks]

    def backward(self, dL_dchi2, stream=None):
        """d(sum dL_dchi2 * chi2)/d theta (float32 [36720]) at the last forward's theta."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        g = dL_dchi2.to(torch.float32).contiguous()
        out = torch.empty(MAP_NCOEF, dtype=torch.float32, device=g.device)
        _check(lib().tpcx_refit_backward(self.tracker._h, ctypes.byref(self.c), _ptr(g), _ptr(out),
                                         self._ws(), self.ws_bytes, ctypes.c_void_p(s.cuda_stream)),
               "tpcx_refit_backward")
        return out


def _make_refit_chi2():
    import torch

    class RefitChi2(torch.autograd.Function):
        """chi2 per track of the map-corrected refit; differentiable in theta.

        forward(theta [36720] float32, job: RefitJob) -> chi2 [n_tracks]
        backward uses the library's hand-written adjoint (tpcx_refit_backward).
        """

        @staticmethod
        def forward(ctx, theta, job):
            ctx.job = job
            th = theta.detach().clone()
            ctx.save_for_backward(th)
            chi2 = job.forward(th).clone()
            ctx.forward_id = job.n_forward
            return chi2

        @staticmethod
        def backward(ctx, grad_chi2):
            (th,) = ctx.saved_tensors
            job = ctx.job
            if job.n_forward != ctx.forward_id:
                # another forward on this job replaced the workspace (corrected
                # clusters, checkpoints, ok flags): redo this node's forward
                job.forward(th)
                ctx.forward_id = job.n_forward
            return job.backward(grad_chi2), None

    return RefitChi2


def refit_chi2(theta, job):
    """Differentiable chi2 per track: RefitChi2.apply(theta, job)."""
    global _RefitChi2
    if "_RefitChi2" not in globals():
        _RefitChi2 = _make_refit_chi2()
    return _RefitChi2.apply(theta, job)
