"""Refit through the distortion map and its hand-written adjoint, on the GPU,
against the FP64 oracle (refit chi2; forward-mode gradient).

The refit input is the oracle's own tracklet list (clusters, rows, seeds), so
no value computed by the HIP path feeds the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import geometry as G

from gpu_helpers import make_tracker

pytestmark = pytest.mark.gpu


def _case(n_primaries=2500, stride=1, seed=5):
    cs = synth.central_event(seed=seed, n_primaries=n_primaries, distortion=synth.RadialDistortion())
    k = oracle.kept_tracklets(oracle.track(cs))
    tk = oracle.select_tracks(k, 20)
    if stride > 1:
        tk = oracle.select_tracks(tk, 20, index=np.arange(0, len(tk["n"]), stride))
    return cs, tk


def _job(cs, tk, tracker=None):
    import torch

    import paper_2601_20569_amd as px
    dev = torch.device("cuda")
    tr = tracker or make_tracker()
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    alpha = G.sector_alpha(cs.unit_sector).astype(np.float32)
    job = px.RefitJob(tr, T(tk["hit_begin"], torch.int64), T(tk["hits"], torch.int32),
                      T(tk["rows"], torch.uint8), T(tk["unit"], torch.int32),
                      T(np.asarray(tk["param"], np.float32), torch.float32), T(cs.y, torch.float32),
                      T(cs.z, torch.float32), T(alpha, torch.float32))
    return job, tr


def _theta(kind, n):
    if kind == "zero":
        return np.zeros(n)
    if kind == "random":
        return np.random.default_rng(3).normal(0.0, 0.05, n)
    from test_refit_oracle import inverse_radial_correction_map
    return inverse_radial_correction_map(synth.RadialDistortion())


@pytest.mark.parametrize("kind", ["zero", "random", "inverse"])
def test_refit_chi2_matches_fp64(kind):
    import torch
    print(f"case: refit forward, theta={kind}", flush=True)
    cs, tk = _case()
    job, _ = _job(cs, tk)
    theta = _theta(kind, oracle.map_ncoef())
    want, ok_ref = oracle.refit(cs, tk, theta)
    chi2 = job.forward(torch.as_tensor(theta, dtype=torch.float32, device="cuda")).cpu().numpy()
    ok = job.ok[:job.n_tracks].cpu().numpy().astype(bool)
    assert len(chi2) > 1000
    np.testing.assert_array_equal(ok, ok_ref)
    rel = np.abs(chi2[ok] - want[ok]) / np.maximum(want[ok], 1.0)
    print(f"refit: {ok.sum()} tracks, max rel {rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-3, rel.max()


def test_refit_without_map_equals_zero_map():
    import torch
    cs, tk = _case(n_primaries=800)
    job, _ = _job(cs, tk)
    a = job.forward(None).cpu().numpy().copy()
    b = job.forward(torch.zeros(oracle.map_ncoef(), dtype=torch.float32, device="cuda")).cpu().numpy()
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("kind", ["zero", "random", "inverse"])
def test_adjoint_matches_fp64_gradient(kind):
    import torch
    print(f"case: refit adjoint, theta={kind}", flush=True)
    cs, tk = _case(stride=4)
    job, _ = _job(cs, tk)
    theta = _theta(kind, oracle.map_ncoef())
    job.forward(torch.as_tensor(theta, dtype=torch.float32, device="cuda"))
    ok = job.ok[:job.n_tracks].cpu().numpy().astype(bool)
    _, ok_ref = oracle.refit(cs, tk, theta)
    w = np.random.default_rng(5).uniform(0.5, 1.5, job.n_tracks) * (ok & ok_ref)
    g = job.backward(torch.as_tensor(w, dtype=torch.float32, device="cuda")).cpu().numpy().astype(np.float64)
    want = oracle.refit_grad(cs, tk, theta, dL_dchi2=w)
    err = np.linalg.norm(g - want) / np.linalg.norm(want)
    assert err < 1e-3, err
    # coefficients without any contributing cluster are exactly zero
    assert (g[want == 0.0] == 0.0).all()
    # element-wise sanity bound (float sums of cancelling contributions): the
    # worst element is reported
    d = np.abs(g - want)
    bound = 2e-2 * np.abs(want) + 2e-3 * np.abs(want).max()
    worst = int(np.argmax(d / bound))
    print(f"relative L2 {err:.2e}; worst element {worst}: gpu {g[worst]:.6g} fp64 {want[worst]:.6g}")
    assert (d <= bound).all()


@pytest.mark.timeout(900)
def test_adjoint_on_the_full_adjoint_workload():
    """The adjoint workload at full size: a central event of 10^4 primaries
    and their secondaries with the radial distortion applied, every tracklet
    of at least 20 clusters refitted through the uncorrected (zero) map.  The
    refit chi2 and ok flags against the FP64 refit, the gradient against the
    FP64 gradient of the same weighted sum."""
    import torch
    print("case: full adjoint workload (central event seed 5, distorted), theta = 0", flush=True)
    cs = synth.central_event(seed=5, distortion=synth.RadialDistortion())
    tk = oracle.select_tracks(oracle.kept_tracklets(oracle.track(cs, n_threads=16)), 20)
    assert len(tk["n"]) > 50000
    job, _ = _job(cs, tk)
    theta = np.zeros(oracle.map_ncoef())
    chi2 = job.forward(torch.as_tensor(theta, dtype=torch.float32, device="cuda")).cpu().numpy()
    ok = job.ok[:job.n_tracks].cpu().numpy().astype(bool)
    want, ok_ref = oracle.refit(cs, tk, theta)
    np.testing.assert_array_equal(ok, ok_ref)
    rel = np.abs(chi2[ok] - want[ok]) / np.maximum(want[ok], 1.0)
    assert rel.max() <= 1e-3, rel.max()
    w = np.random.default_rng(6).uniform(0.5, 1.5, job.n_tracks) * ok
    g = job.backward(torch.as_tensor(w, dtype=torch.float32, device="cuda")).cpu().numpy().astype(np.float64)
    want_g = oracle.refit_grad(cs, tk, theta, dL_dchi2=w)
    err = np.linalg.norm(g - want_g) / np.linalg.norm(want_g)
    print(f"{ok.sum()} tracks refitted, chi2 max rel {rel.max():.2e}, gradient relative L2 {err:.2e}", flush=True)
    assert err < 1e-3, err
    assert (g[want_g == 0.0] == 0.0).all()
    d = np.abs(g - want_g)
    assert (d <= 2e-2 * np.abs(want_g) + 2e-3 * np.abs(want_g).max()).all()


def test_adjoint_is_deterministic_and_linear_in_weights():
    import torch
    cs, tk = _case(n_primaries=1500)
    job, _ = _job(cs, tk)
    th = torch.as_tensor(_theta("random", oracle.map_ncoef()), dtype=torch.float32, device="cuda")
    job.forward(th)
    w = torch.ones(job.n_tracks, dtype=torch.float32, device="cuda") * job.ok[:job.n_tracks].float()
    a = job.backward(w).cpu().numpy()
    b = job.backward(w).cpu().numpy()
    np.testing.assert_array_equal(a, b)
    c = job.backward(2.0 * w).cpu().numpy()
    np.testing.assert_allclose(c, 2.0 * a, rtol=1e-6, atol=1e-6 * np.abs(a).max())


def test_autograd_function_uses_the_adjoint():
    import torch

    import paper_2601_20569_amd as px
    cs, tk = _case(n_primaries=1500)
    job, _ = _job(cs, tk)
    theta = torch.as_tensor(_theta("random", oracle.map_ncoef()), dtype=torch.float32,
                            device="cuda").requires_grad_(True)
    chi2 = px.refit_chi2(theta, job)
    ok = job.ok[:job.n_tracks].float()
    loss = (chi2 * ok).sum()
    (g,) = torch.autograd.grad(loss, theta)
    want = job.backward(ok)
    np.testing.assert_array_equal(g.cpu().numpy(), want.cpu().numpy())


def test_autograd_backward_after_another_forward_on_the_job():
    """Two refit_chi2 nodes on one job, the second forward run before the first
    node's backward: the first node's gradient is its own theta's, not the
    workspace's last state."""
    import torch

    import paper_2601_20569_amd as px
    cs, tk = _case(n_primaries=800)
    job, _ = _job(cs, tk)
    rng = np.random.default_rng(4)
    t1 = torch.as_tensor(rng.normal(0.0, 0.05, oracle.map_ncoef()), dtype=torch.float32, device="cuda")
    t2 = torch.as_tensor(rng.normal(0.0, 0.05, oracle.map_ncoef()), dtype=torch.float32, device="cuda")
    job.forward(t1)
    ok = job.ok[:job.n_tracks].float().clone()
    want1 = job.backward(ok).cpu().numpy()
    job.forward(t2)
    ok2 = job.ok[:job.n_tracks].float().clone()
    want2 = job.backward(ok2).cpu().numpy()
    assert not np.array_equal(want1, want2)
    a = t1.clone().requires_grad_(True)
    b = t2.clone().requires_grad_(True)
    c1 = px.refit_chi2(a, job)
    c2 = px.refit_chi2(b, job)  # replaces the job's workspace
    (g1,) = torch.autograd.grad((c1 * ok).sum(), a)
    np.testing.assert_array_equal(g1.cpu().numpy(), want1)
    (g2,) = torch.autograd.grad((c2 * ok2).sum(), b)
    np.testing.assert_array_equal(g2.cpu().numpy(), want2)


def test_adjoint_matches_central_differences_of_fp64_refit():
    """Directional derivatives of sum_t w_t chi2_t: the GPU adjoint against
    central finite differences (h = 1e-3 cm) of the FP64 oracle refit."""
    import torch
    print("case: adjoint vs central differences, 6 directions", flush=True)
    cs, tk = _case(n_primaries=1500, stride=3)
    job, _ = _job(cs, tk)
    rng = np.random.default_rng(21)
    theta = rng.normal(0.0, 0.05, oracle.map_ncoef())
    job.forward(torch.as_tensor(theta, dtype=torch.float32, device="cuda"))
    ok = job.ok[:job.n_tracks].cpu().numpy().astype(bool)
    _, ok_ref = oracle.refit(cs, tk, theta)
    w = rng.uniform(0.5, 1.5, job.n_tracks) * (ok & ok_ref)
    g = job.backward(torch.as_tensor(w, dtype=torch.float32, device="cuda")).cpu().numpy().astype(np.float64)
    h = 1e-3
    for _ in range(6):
        v = rng.normal(size=len(theta))
        v /= np.linalg.norm(v)
        cp, okp = oracle.refit(cs, tk, theta + h * v)
        cm, okm = oracle.refit(cs, tk, theta - h * v)
        assert (okp == ok_ref).all() and (okm == ok_ref).all()
        fd = float(w @ (cp - cm)) / (2 * h)
        print(f"directional derivative: gpu {g @ v:.6g} fd {fd:.6g}")
        assert abs(g @ v - fd) <= 1e-3 * np.linalg.norm(g), (g @ v, fd)
