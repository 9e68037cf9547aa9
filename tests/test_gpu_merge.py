"""Track merging on the GPU (tpcx_merge) against the oracle (oracle.merge),
bit for bit: the links (prev, next) and chain roots of every track.  Inputs
are truth segments and the oracle's own selected tracklets (no value of the
HIP path feeds the oracle): segments split inside a sector, crossing into the
next sector and across the central electrode, the selected tracklets of the
central event (36 units, with the electrode step), time-frame units, and
random inputs with exact chi2 ties."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import geometry as G

from gpu_helpers import make_tracker
from test_merge_oracle import as_tracks, helix_state, segments

pytestmark = pytest.mark.gpu


def _gpu(tk, nbr, n_units, **kw):
    import torch
    dev = torch.device("cuda")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    tr = make_tracker()
    f = dict(oracle.MERGE_DEFAULTS, **kw)
    g = tr.merge(T(tk["unit"], torch.int32), T(np.asarray(tk["param"], np.float32), torch.float32),
                 T(np.asarray(tk["xref"], np.float32), torch.float32), T(tk["r_in"], torch.int32),
                 T(tk["r_out"], torch.int32), T(nbr, torch.int32), n_units, x_m=f["x_m"], tol=f["tol"],
                 chi2_cut=f["chi2_cut"], cross_electrode=f["cross_electrode"], half_opening=G.HALF_OPENING_RAD)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items() if k != "_ws"}


def _check(tk, nbr, n_units, name, **kw):
    print(f"case: {name}, {len(tk['unit'])} tracks", flush=True)
    g = _gpu(tk, nbr, n_units, **kw)
    r = oracle.merge(tk, nbr, n_units, **kw)
    for k in ("prev", "next", "root"):
        np.testing.assert_array_equal(g[k], r[k], err_msg=k)
    links = int((r["next"] >= 0).sum())
    print(f"  {links} links", flush=True)
    return links


def test_merge_truth_segments():
    cs = synth.exact_tracks(62, n_tracks=14, pt_range=(0.8, 8.0))
    assert _check(as_tracks(segments(cs, split=(40, 6))), oracle.unit_neighbours([0]), 1, "split segments") >= 10
    rng = np.random.default_rng(7)
    n = 60
    phi = rng.uniform(math.radians(8.0), math.radians(32.0), n)
    pt = np.exp(rng.uniform(math.log(0.3), math.log(1.0), n))
    tr = synth.events.Tracks(np.zeros(n), np.zeros(n), np.zeros(n), pt, phi, rng.uniform(0.05, 0.5, n),
                             rng.choice([-1.0, 1.0], n), np.zeros(n))
    cs = synth.build_clusters(tr, [0, 1], 5, smear_sigma=0.0, noise_frac=0.0)
    assert _check(as_tracks(segments(cs)), oracle.unit_neighbours([0, 1]), 2, "sector crossings") >= 10
    n = 6
    phi = rng.uniform(math.radians(3.0), math.radians(17.0), n)
    tr = synth.events.Tracks(np.zeros(n), np.zeros(n), np.full(n, 12.0), np.full(n, 5.0), phi,
                             np.full(n, -0.1), rng.choice([-1.0, 1.0], n), np.zeros(n))
    x = G.row_x()
    a0 = float(G.sector_alpha(0))
    segs = []
    for t in range(n):
        states = [helix_state(tr, t, a0, xr) for xr in x]
        k = int(np.argmax(np.array([s[1] for s in states]) < 0))
        segs.append(dict(unit=0, r_in=0, r_out=k - 1, param=states[0], xref=float(x[0])))
        segs.append(dict(unit=1, r_in=k, r_out=len(x) - 1, param=states[k], xref=float(x[k])))
    segs.sort(key=lambda s: s["unit"])
    assert _check(as_tracks(segs), oracle.unit_neighbours([0, 18]), 2, "electrode crossings") == n


def _selected(cs, unit_group=None):
    k = oracle.kept_tracklets(oracle.track(cs, n_threads=16))
    keep, _ = oracle.select(k, cs.n_clusters)
    idx = np.nonzero(keep)[0]
    hb = k["hit_begin"]
    return dict(unit=k["unit"][idx].astype(np.int32), param=k["param"][idx], xref=k["xref"][idx],
                r_in=np.array([k["rows"][hb[i]] for i in idx], np.int32),
                r_out=np.array([k["rows"][hb[i + 1] - 1] for i in idx], np.int32))


def test_merge_selected_tracklets_of_the_central_event():
    cs = synth.central_event(seed=2)
    tk = _selected(cs)
    nbr = oracle.unit_neighbours(cs.unit_sector)
    assert _check(tk, nbr, cs.n_units, "central event, selected tracklets") > 100


def test_merge_timeframe_units():
    from types import SimpleNamespace
    cs = synth.timeframe_slice(seed=3004, n_collisions=24, device="cuda", truth=False)
    R = G.N_ROWS
    u0, u1 = 0, 4  # sectors 0..3 of side A: three boundaries
    lo, hi = int(cs.row_begin[u0 * R]), int(cs.row_begin[u1 * R])
    cu = SimpleNamespace(n_units=u1 - u0, row_begin=cs.row_begin[u0 * R:u1 * R + 1] - lo,
                         y=np.asarray(cs.y[lo:hi]), z=np.asarray(cs.z[lo:hi]), n_clusters=hi - lo)
    tk = _selected(cu)
    nbr = oracle.unit_neighbours(cs.unit_sector[u0:u1])
    # the drift coordinate of a time frame is not z: no electrode step
    _check(tk, nbr, cu.n_units, "time-frame units 0..3", cross_electrode=False)


def test_merge_random_inputs_with_ties():
    rng = np.random.default_rng(12)
    for case in range(6):
        n_units = 4
        sectors = np.array([0, 1, 18, 19])
        n = 3000
        unit = np.sort(rng.integers(0, n_units, n)).astype(np.int32)
        base = np.array([0.0, 0.0, 0.0, 0.2, 0.5])
        param = base + rng.normal(0, 1, (n, 5)) * np.array([8.0, 40.0, 0.02, 0.01, 0.05])
        param[1::3] = param[0::3][:len(param[1::3])]  # exact ties
        r_in = rng.integers(0, 150, n).astype(np.int32)
        r_out = np.minimum(151, r_in + rng.integers(2, 60, n)).astype(np.int32)
        tk = dict(unit=unit, param=param, xref=G.row_x()[r_in].astype(np.float64), r_in=r_in, r_out=r_out)
        _check(tk, oracle.unit_neighbours(sectors), n_units, f"random case {case}")
