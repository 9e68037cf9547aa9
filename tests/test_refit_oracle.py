"""Pins of the refit oracle: the B-spline distortion map, the refit chi2, and
its FP64 gradient with respect to the map coefficients.

* basis: weights equal to products of scipy's cubic B-spline basis elements,
  partition of unity (periodic phi; interior r and z), exact reproduction of
  linear functions, linearity of the map in theta;
* refit: zero chi2 for exact helices seeded with the truth, chi2/ndf = 1 on
  smeared tracks, and a least-squares map fitted to the exact inverse of the
  generator's radial distortion removes the distortion's chi2;
* gradient (forward-mode dual numbers): central finite differences of the
  FP64 refit (h = 1e-3 cm) on >= 512 populated coefficients and 16 random
  directions; coefficients whose support holds no cluster are exactly 0.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import geometry as G

NPHI, NR, NZ = 36, 17, 20
R_NODES = 85.0 + 10.0 * np.arange(NR)
Z_NODES = -250.0 + np.arange(NZ) * 500.0 / 19.0


def coef(comp, i, j, k):
    return ((comp * NPHI + i) * NR + j) * NZ + k


def test_basis_partition_of_unity_and_linear_reproduction():
    rng = np.random.default_rng(1)
    assert oracle.map_ncoef() == 3 * NPHI * NR * NZ == 36720
    for _ in range(300):
        phi = rng.uniform(-10, 10)
        r = rng.uniform(R_NODES[1], R_NODES[-2])
        z = rng.uniform(Z_NODES[1], Z_NODES[-2])
        idx, w = oracle.map_basis(r, phi, z)
        assert len(w) == 64 and (w > 0).all()
        assert abs(w.sum() - 1.0) < 1e-12
        # linear functions of r and z are reproduced from nodal values
        a, b, c = rng.normal(size=3)
        rr = R_NODES[idx[:, 1]]
        zz = Z_NODES[idx[:, 2]]
        assert abs((w * (a + b * rr + c * zz)).sum() - (a + b * r + c * z)) < 1e-9
    # outside the node ranges the basis is cut, not renormalised
    idx, w = oracle.map_basis(80.0, 0.3, 0.0)
    assert w.sum() < 1.0


def test_basis_weights_are_scipy_cubic_bspline_products():
    """Each weight is the product of three uniform cubic B-spline basis
    elements (scipy's definition from the knots), one per coordinate, centred
    on the node, with phi periodic; and every node whose product is non-zero
    is listed.  Partition of unity and linear reproduction alone would also
    admit linear (hat) B-splines: this pins the order."""
    from scipy.interpolate import BSpline
    cubic = BSpline.basis_element(np.arange(-2.0, 3.0), extrapolate=False)

    def b(t):
        v = cubic(t)
        return 0.0 if np.isnan(v) else float(v)

    dphi = 2.0 * math.pi / NPHI
    dz = 500.0 / 19.0
    rng = np.random.default_rng(5)
    for _ in range(200):
        phi = rng.uniform(-10, 10)
        r = rng.uniform(70.0, 260.0)
        z = rng.uniform(-280.0, 280.0)
        idx, w = oracle.map_basis(r, phi, z)
        got = {tuple(int(v) for v in row): wt for row, wt in zip(idx, w)}
        want = {}
        for i in range(NPHI):
            tp = math.remainder(phi - i * dphi, 2.0 * math.pi) / dphi
            bi = b(tp)
            if bi == 0.0:
                continue
            for j in range(NR):
                bj = b((r - R_NODES[j]) / 10.0)
                if bj == 0.0:
                    continue
                for k in range(NZ):
                    bk = b((z - Z_NODES[k]) / dz)
                    if bk != 0.0:
                        want[(i, j, k)] = bi * bj * bk
        assert set(got) == set(want)
        for key, wt in want.items():
            assert abs(got[key] - wt) < 1e-12


def test_map_is_linear_in_theta_and_matches_basis():
    rng = np.random.default_rng(2)
    n = oracle.map_ncoef()
    t1, t2 = rng.normal(size=n), rng.normal(size=n)
    for _ in range(50):
        r, phi, z = rng.uniform(85, 245), rng.uniform(0, 7), rng.uniform(-250, 250)
        d = oracle.map_eval(t1 + 2.0 * t2, r, phi, z)
        np.testing.assert_allclose(d, oracle.map_eval(t1, r, phi, z) + 2.0 * oracle.map_eval(t2, r, phi, z),
                                   rtol=1e-12, atol=1e-12)
        idx, w = oracle.map_basis(r, phi, z)
        for comp in range(3):
            want = sum(t1[coef(comp, *ix)] * ww for ix, ww in zip(idx, w))
            assert abs(oracle.map_eval(t1, r, phi, z)[comp] - want) < 1e-12
    assert (oracle.map_eval(None, 100.0, 1.0, 0.0) == 0).all()


def truth_tracklets(cs):
    """One tracklet per particle: all its clusters sorted by row, seeded with
    the truth direction and curvature at the innermost cluster."""
    rows = cs.row_of()
    tr = cs.tracks
    hits, rws, seeds, nn = [], [], [], []
    for t in np.unique(cs.truth_track[cs.truth_track >= 0]):
        idx = np.nonzero(cs.truth_track == t)[0]
        if len(idx) < 20:
            continue
        idx = idx[np.argsort(rows[idx])]
        j = idx[0]
        a0 = float(G.sector_alpha(cs.unit_sector[0]))
        phi = tr.phi[t] - tr.q[t] * cs.truth_psi[j]
        seeds.append([cs.y[j], cs.z[j], math.sin(phi - a0), tr.tanl[t], tr.q[t] / tr.pt[t]])
        hits.append(idx)
        rws.append(rows[idx])
        nn.append(len(idx))
    hb = np.zeros(len(nn) + 1, np.int64)
    hb[1:] = np.cumsum(nn)
    return dict(hit_begin=hb, hits=np.concatenate(hits).astype(np.int32),
                rows=np.concatenate(rws).astype(np.uint8), unit=np.zeros(len(nn), np.int32),
                param=np.array(seeds), n=np.array(nn))


def test_refit_of_exact_helices_has_zero_chi2():
    cs = synth.exact_tracks(41, n_tracks=10, pt_range=(0.5, 10.0))
    tk = truth_tracklets(cs)
    chi2, ok = oracle.refit(cs, tk)
    assert ok.all() and len(chi2) >= 8
    assert (chi2 < 1e-6).all(), chi2


def test_refit_chi2_per_ndf_is_one_on_smeared_tracks():
    ratios = []
    for seed in range(6):
        tr = synth.exact_tracks(500 + seed, n_tracks=20, pt_range=(1.0, 10.0)).tracks
        cs = synth.build_clusters(tr, [0], seed + 3, smear_sigma=0.1, noise_frac=0.0)
        tk = truth_tracklets(cs)
        chi2, ok = oracle.refit(cs, tk)
        ratios += list(chi2[ok] / (2 * tk["n"][ok] - 5))
    assert len(ratios) > 80
    assert abs(np.mean(ratios) - 1.0) < 0.05


def inverse_radial_correction_map(dist):
    """theta whose delta-r component is the least-squares fit of the exact
    inverse of the radial distortion (r_true = r_meas + delta): a 1-D fit over
    the r nodes, copied to every phi and z node (the phi basis sums to one,
    and so does the z basis away from the ends)."""
    r = np.linspace(85.0, 250.0, 2000)
    rt = r.copy()
    for _ in range(80):
        rt = r + dist.shift(rt)
    A = np.zeros((len(r), NR))
    for q, rr in enumerate(r):
        idx, w = oracle.map_basis(rr, 0.123, 0.0)
        for ix, ww in zip(idx, w):
            A[q, ix[1]] += ww
    # the phi and z weights of one point sum to one here: A holds the r weights
    a, *_ = np.linalg.lstsq(A, rt - r, rcond=None)
    theta = np.zeros(oracle.map_ncoef())
    for i in range(NPHI):
        for j in range(NR):
            for k in range(NZ):
                theta[coef(0, i, j, k)] = a[j]
    return theta


def test_fitted_inverse_map_removes_the_distortion():
    dist = synth.RadialDistortion()
    tr = synth.exact_tracks(61, n_tracks=12, pt_range=(1.0, 10.0), eta_range=(0.05, 0.6)).tracks
    cs = synth.build_clusters(tr, [0], 9, smear_sigma=0.0, noise_frac=0.0, distortion=dist)
    tk = truth_tracklets(cs)
    theta = inverse_radial_correction_map(dist)
    c0, ok0 = oracle.refit(cs, tk)
    c1, ok1 = oracle.refit(cs, tk, theta)
    good = ok0 & ok1
    assert good.sum() >= 8
    # the cubic B-spline misses the 1/r^2 shape by up to ~0.3 cm at the inner
    # edge, so a residual chi2 remains (observed reduction ~80x)
    assert np.median(c0[good]) > 30.0 * np.median(c1[good]), (np.median(c0[good]), np.median(c1[good]))


@pytest.fixture(scope="module")
def grad_case():
    cs = synth.central_event(seed=5, n_primaries=1500, distortion=synth.RadialDistortion())
    k = oracle.kept_tracklets(oracle.track(cs))
    tk = oracle.select_tracks(k, 20)
    sub = oracle.select_tracks(tk, 20, index=np.arange(0, len(tk["n"]), 6))
    rng = np.random.default_rng(7)
    theta = rng.normal(0.0, 0.05, oracle.map_ncoef())
    _, ok = oracle.refit(cs, sub, theta)
    w = ok.astype(float) * rng.uniform(0.5, 1.5, len(ok))
    g = oracle.refit_grad(cs, sub, theta, dL_dchi2=w)
    return cs, sub, theta, w, ok, g


def _loss(cs, sub, theta, w, ok_ref):
    chi2, ok = oracle.refit(cs, sub, theta)
    assert (ok == ok_ref).all()
    return float((w * chi2).sum())


def test_gradient_matches_central_differences(grad_case):
    cs, sub, theta, w, ok, g = grad_case
    nz = np.nonzero(g)[0]
    rms = math.sqrt(float(np.mean(g[nz] ** 2)))
    rng = np.random.default_rng(11)
    pick = rng.choice(nz, 512, replace=False)
    h = 1e-3
    for i in pick:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (_loss(cs, sub, tp, w, ok) - _loss(cs, sub, tm, w, ok)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * abs(g[i]) + 1e-6 * rms, (i, fd, g[i])


def test_gradient_directional_derivatives(grad_case):
    cs, sub, theta, w, ok, g = grad_case
    rng = np.random.default_rng(12)
    h = 1e-3
    for _ in range(16):
        v = rng.normal(size=len(theta))
        v /= np.linalg.norm(v)
        fd = (_loss(cs, sub, theta + h * v, w, ok) - _loss(cs, sub, theta - h * v, w, ok)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-5 * np.linalg.norm(g)


def test_gradient_is_zero_where_no_cluster_contributes(grad_case):
    cs, sub, theta, w, ok, g = grad_case
    support = np.zeros(len(g), bool)
    rows = sub["rows"]
    xr = G.row_x().astype(np.float64)
    alpha = G.sector_alpha(cs.unit_sector)
    for t in range(len(sub["n"])):
        if w[t] == 0:
            continue
        for q in range(sub["hit_begin"][t], sub["hit_begin"][t + 1]):
            x, y, z = xr[rows[q]], float(cs.y[sub["hits"][q]]), float(cs.z[sub["hits"][q]])
            idx, _ = oracle.map_basis(math.hypot(x, y), alpha[sub["unit"][t]] + math.atan2(y, x), z)
            for ix in idx:
                for comp in range(3):
                    support[coef(comp, *ix)] = True
    assert (g[~support] == 0.0).all()
    assert support.sum() > 1000
