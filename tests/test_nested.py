"""The device nested-sampling driver against the nested-sampling oracle.

Both consume the same candidate stream (random numbers are inputs, drawn by one seeded numpy
generator per side) and the same analytic likelihood, so the dead-point sequence, the prior
volumes and the evidence must agree to rounding. The radial likelihood has no ties, so the dead
points' coordinates must agree too. The CPU cases run the driver on host tensors; the GPU cases
run the same comparison on the device and a full run on the GW likelihood.
"""
import math
import warnings

import numpy as np
import pytest
import torch

from oracle import ns_oracle as ns
from paper_1909_11873_amd import nested
from tests.test_ns_oracle import ball_proposer, prior_proposer, radial


def torch_radial(s):
    return lambda th: -((th - 0.5) ** 2).sum(dim=1) / (2 * s * s)


def wrap(numpy_proposer, dev):
    """The same proposal function on device tensors."""
    def propose(it, live_u, live_l):
        c = numpy_proposer(it, live_u.cpu().numpy(), live_l.cpu().numpy())
        return torch.tensor(c, dtype=torch.float64, device=dev)
    return propose


def compare(dev, kind, n, K=60, d=3, s=0.06, eps=0.05, seed=21):
    live = np.random.default_rng(seed).random((K, d))
    mk = (lambda: ball_proposer(d, n, s, seed + 1)) if kind == "ball" else (lambda: prior_proposer(d, n, seed + 1))
    ref = ns.run(radial(s), live, mk(), eps=eps)
    smp = nested.ParallelNestedSampler(torch_radial(s), d, K, n, device=dev, proposal=wrap(mk(), dev),
                                       check_every=3)
    got = smp.run(eps=eps, live_u=torch.tensor(live))
    assert got.niter == ref["niter"]
    np.testing.assert_array_equal(got.n_accepted, ref["n_accepted"])
    np.testing.assert_allclose(got.logl, ref["logl"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(got.u, ref["u"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(got.log_x[:-1], ref["log_x"][:-1], rtol=0, atol=1e-10)
    np.testing.assert_allclose(got.log_dx, ref["log_dx"], rtol=0, atol=1e-10)
    assert got.logz == pytest.approx(ref["logz"], abs=1e-10)
    return got, ref


@pytest.mark.parametrize("kind,n", [("ball", 1), ("ball", 16), ("ball", 500), ("prior", 64), ("prior", 1000)])
def test_driver_matches_oracle_on_host(kind, n):
    compare(torch.device("cpu"), kind, n)


def test_driver_paper_volume_option_matches_oracle():
    d, K, s, n = 2, 30, 0.1, 50
    live = np.random.default_rng(3).random((K, d))
    ref = ns.run(radial(s), live, ball_proposer(d, n, s, 4), eps=0.1, volume="paper")
    got = nested.ParallelNestedSampler(torch_radial(s), d, K, n, device="cpu", volume="paper",
                                       proposal=wrap(ball_proposer(d, n, s, 4), "cpu")).run(
        eps=0.1, live_u=torch.tensor(live))
    np.testing.assert_allclose(got.log_x[:-1], ref["log_x"][:-1], atol=1e-10)
    assert got.logz == pytest.approx(ref["logz"], abs=1e-10)


def test_driver_ellipsoid_proposal_on_host():
    """The driver's own bounding-ellipsoid proposal: evidence and moments of the radial Gaussian."""
    d, K, s = 3, 300, 0.07
    smp = nested.ParallelNestedSampler(torch_radial(s), d, K, 512, device="cpu", seed=5)
    res = smp.run(eps=0.01)
    z_true = d * math.log(math.sqrt(2 * math.pi) * s * math.erf(0.5 / (s * math.sqrt(2))))
    assert abs(res.logz - z_true) < 4 * res.logz_err + 0.05
    w = np.exp(res.log_w)
    var = np.sum(w[:, None] * (res.u - np.sum(w[:, None] * res.u, 0)) ** 2, 0)
    np.testing.assert_allclose(var, s * s, rtol=0.25)
    nd = len(res.logl) - K
    assert np.all(np.diff(res.logl[:nd]) >= 0)


def test_gmc_proposal_on_host():
    """Gradient-guided walks (Galilean Monte Carlo) as the proposal: evidence and moments of the
    radial Gaussian, with the analytic gradient standing in for the library's adjoint."""
    d, K, s = 3, 200, 0.07
    lg = lambda th: (torch_radial(s)(th), -(th - 0.5) / (s * s))
    smp = nested.ParallelNestedSampler(torch_radial(s), d, K, 256, device="cpu", seed=7, proposal="gmc",
                                       loglike_grad=lg, gmc_steps=6)
    res = smp.run(eps=0.01)
    z_true = d * math.log(math.sqrt(2 * math.pi) * s * math.erf(0.5 / (s * math.sqrt(2))))
    assert abs(res.logz - z_true) < 4 * res.logz_err + 0.1, (res.logz, z_true, res.logz_err)
    w = np.exp(res.log_w)
    var = np.sum(w[:, None] * (res.u - np.sum(w[:, None] * res.u, 0)) ** 2, 0)
    np.testing.assert_allclose(var, s * s, rtol=0.3)
    assert res.ncall > K + 256 * res.niter     # the walks' own evaluations are counted


def test_gmc_correlated_gaussian_on_host():
    """A normalised, strongly correlated Gaussian (rho = 0.98) inside the cube: ln Z = 0."""
    s, rho = 0.05, 0.98
    cov = s * s * torch.tensor([[1.0, rho, 0.0], [rho, 1.0, 0.0], [0.0, 0.0, 1.0]], dtype=torch.float64)
    prec = torch.linalg.inv(cov)
    norm = -0.5 * math.log((2 * math.pi) ** 3 * float(torch.linalg.det(cov)))

    def ll(th):
        x = th - 0.5
        return norm - 0.5 * ((x @ prec) * x).sum(1)

    lg = lambda th: (ll(th), -((th - 0.5) @ prec))
    res = nested.ParallelNestedSampler(ll, 3, 300, 128, device="cpu", seed=9, proposal="gmc", loglike_grad=lg,
                                       gmc_steps=10).run(eps=0.01)
    assert abs(res.logz) < 4 * res.logz_err + 0.1, (res.logz, res.logz_err)
    w = np.exp(res.log_w)
    m = np.sum(w[:, None] * res.u, 0)
    c = np.einsum("i,ij,ik->jk", w, res.u - m, res.u - m)
    assert c[0, 1] / math.sqrt(c[0, 0] * c[1, 1]) == pytest.approx(rho, abs=0.02)


def two_balls(p):
    """Membership in a region whose lines need not cross it in one piece: two balls in the cube."""
    inc = ((p >= 0.0) & (p <= 1.0)).all(-1)
    return inc & ((((p - 0.3) ** 2).sum(-1) < 0.2 ** 2) | (((p - 0.7) ** 2).sum(-1) < 0.15 ** 2))


def neal_slice_move(x0, dirn, unif, m, inside):
    """Neal's stepping-out and shrinkage, one chain at a time, with the same uniform numbers."""
    r = unif[0]
    lo0, hi0 = -r, 1.0 - r
    sl = sr = 0
    if m > 1:
        jl = math.floor(m * unif[1])
        jr = m - 1 - jl
        while sl < jl and inside(x0 + (lo0 - sl) * dirn):
            sl += 1
        while sr < jr and inside(x0 + (hi0 + sr) * dirn):
            sr += 1
    lo, hi = lo0 - sl, hi0 + sr
    for k in range(nested.SLICE_MAX_DRAWS):
        t = lo + unif[2 + k] * (hi - lo)
        p = x0 + t * dirn
        if inside(p):
            return p, True
        if t < 0.0:
            lo = t
        else:
            hi = t
    return x0, False


@pytest.mark.parametrize("m", [1, 4])
def test_slice_move_is_the_sequential_procedure(m):
    """The batched slice move (ends and shrinkage draws evaluated ahead, in groups) returns
    exactly what the sequential procedure returns with the same random numbers."""
    rng = np.random.default_rng(11 + m)
    n, d = 400, 3
    x = np.where(rng.random((3 * n, 1)) < 0.5, 0.3, 0.7) + 0.05 * rng.standard_normal((3 * n, d))
    x = x[two_balls(torch.tensor(x)).numpy()][:n]
    assert len(x) == n
    dirn = rng.standard_normal((n, d)) + np.where(rng.random((n, 1)) < 0.5, 3.0, 0.0)   # half near the diagonal
    dirn *= (0.02 + 0.8 * rng.random((n, 1))) / np.linalg.norm(dirn, axis=1, keepdims=True)
    unif = rng.random((2 + nested.SLICE_MAX_DRAWS, n))
    got, moved = nested.slice_move(torch.tensor(x), torch.tensor(dirn), torch.tensor(unif), m, two_balls)
    inside_np = lambda p: bool(two_balls(torch.tensor(p)))
    for i in range(n):
        ref, ok = neal_slice_move(x[i], dirn[i], unif[:, i], m, inside_np)
        assert bool(moved[i]) == ok
        np.testing.assert_array_equal(got[i].numpy(), ref)
    assert bool(moved.all())
    assert (np.linalg.norm(got.numpy() - x, axis=1) > 0).all()
    # some lines left one ball for the other
    assert ((np.linalg.norm(x - 0.3, axis=1) < 0.2) != (np.linalg.norm(got.numpy() - 0.3, axis=1) < 0.2)).any()


def test_slice_moves_keep_the_region_uniform():
    """Uniform points in a ball stay uniform under slice moves: (r / R)^3 stays U(0, 1) and the
    direction stays isotropic."""
    from scipy import stats
    rng = np.random.default_rng(5)
    n, d, R = 20000, 3, 0.3
    v = rng.standard_normal((n, d))
    x = 0.5 + R * v / np.linalg.norm(v, axis=1, keepdims=True) * rng.random((n, 1)) ** (1.0 / d)
    inside = lambda p: ((p - 0.5) ** 2).sum(-1) < R * R
    xt = torch.tensor(x)
    for step in range(3):
        dirn = torch.tensor(rng.standard_normal((n, d)))
        dirn = 0.25 * dirn / dirn.norm(dim=1, keepdim=True)
        xt, moved = nested.slice_move(xt, dirn, torch.tensor(rng.random((2 + nested.SLICE_MAX_DRAWS, n))), 4, inside)
        assert bool(moved.all())
    y = xt.numpy() - 0.5
    r = np.linalg.norm(y, axis=1)
    assert r.max() < R
    assert stats.kstest((r / R) ** 3, "uniform").pvalue > 1e-3
    np.testing.assert_allclose(y.mean(0), 0.0, atol=4 * R / math.sqrt(5 * n))
    assert stats.kstest(y[:, 2] / r, "uniform", args=(-1, 2)).pvalue > 1e-3


def test_slice_proposal_on_host():
    """Slice-sampling walks as the proposal: the normalised correlated Gaussian (ln Z = 0) and its
    correlation; every candidate lies inside the contour, so every candidate is accepted."""
    s, rho = 0.05, 0.98
    cov = s * s * torch.tensor([[1.0, rho, 0.0], [rho, 1.0, 0.0], [0.0, 0.0, 1.0]], dtype=torch.float64)
    prec = torch.linalg.inv(cov)
    norm = -0.5 * math.log((2 * math.pi) ** 3 * float(torch.linalg.det(cov)))

    def ll(th):
        x = th - 0.5
        return norm - 0.5 * ((x @ prec) * x).sum(1)

    res = nested.ParallelNestedSampler(ll, 3, 300, 128, device="cpu", seed=9, proposal="slice").run(eps=0.01)
    assert abs(res.logz) < 4 * res.logz_err + 0.1, (res.logz, res.logz_err)
    assert np.all(res.n_accepted == 128)
    w = np.exp(res.log_w)
    m = np.sum(w[:, None] * res.u, 0)
    c = np.einsum("i,ij,ik->jk", w, res.u - m, res.u - m)
    assert c[0, 1] / math.sqrt(c[0, 0] * c[1, 1]) == pytest.approx(rho, abs=0.02)


def test_slice_chains_that_never_move_are_rejected():
    """A contour that no shrinkage draw can hit (the likelihood is finite only at the live points
    themselves): every move of every chain gives up, so each chain still sits on the live point
    it started from. Such chains come back outside the unit cube (rejected), not as copies of
    live points; with a likelihood that chains can move in, none is."""
    d, K, n = 2, 40, 64
    live = torch.rand(K, d, dtype=torch.float64, generator=torch.Generator().manual_seed(3))

    def needle(th):
        hit = (th[:, None, :] == live[None]).all(-1).any(-1)
        return torch.where(hit, torch.zeros(th.shape[0], dtype=torch.float64),
                           torch.full((th.shape[0],), -math.inf, dtype=torch.float64))

    smp = nested.ParallelNestedSampler(needle, d, K, n, device="cpu", seed=4, proposal="slice", slice_steps=2)
    cand = smp._slice(live, torch.zeros(K, dtype=torch.float64))
    assert cand.shape == (n, d)
    assert bool(((cand < 0.0) | (cand > 1.0)).any(1).all())          # all outside the cube
    # an ordinary contour: every chain moves and stays inside the cube
    smp2 = nested.ParallelNestedSampler(lambda th: -((th - 0.5) ** 2).sum(1), d, K, n, device="cpu", seed=4,
                                        proposal="slice", slice_steps=2)
    lv = 0.5 + 0.1 * (live - 0.5)
    ll = -((lv - 0.5) ** 2).sum(1)
    order = torch.argsort(ll)
    cand2 = smp2._slice(lv[order], ll[order])
    assert bool(((cand2 >= 0.0) & (cand2 <= 1.0)).all())


def test_slice_evidence_scatter_matches_its_quoted_error():
    """Ten independent slice-walk runs on a normalised 4-D Gaussian (ln Z = 0): their mean is
    within three standard errors of 0, and their scatter agrees with the sqrt(H/K) error each run
    quotes (within the spread a sample of ten allows)."""
    d, s = 4, 0.05
    norm = -d * math.log(math.sqrt(2 * math.pi) * s)
    ll = lambda th: norm - ((th - 0.5) ** 2).sum(1) / (2 * s * s)
    zs, es = [], []
    for seed in range(10):
        res = nested.ParallelNestedSampler(ll, d, 150, 64, device="cpu", seed=seed, proposal="slice").run(eps=0.01)
        zs.append(res.logz)
        es.append(res.logz_err)
    err = float(np.median(es))
    assert abs(np.mean(zs)) < 3 * err / math.sqrt(len(zs)) + 0.01, zs
    assert 0.5 * err < np.std(zs, ddof=1) < 1.6 * err, (np.std(zs, ddof=1), err)


def test_importance_logz_on_a_normalised_gaussian():
    """The importance-sampling check itself: ln Z = 0 for a normalised Gaussian inside the cube."""
    s = 0.05
    cov = s * s * np.array([[1.0, 0.9, 0.0], [0.9, 1.0, 0.0], [0.0, 0.0, 1.0]])
    prec = torch.tensor(np.linalg.inv(cov))
    norm = -0.5 * math.log((2 * math.pi) ** 3 * np.linalg.det(cov))
    ll = lambda th: norm - 0.5 * (((th - 0.5) @ prec) * (th - 0.5)).sum(1)
    post = np.random.default_rng(1).multivariate_normal(np.full(3, 0.5), cov, size=4000)
    lz, rel, ess = nested.importance_logz(post, ll, lambda u: u, torch.device("cpu"), ncomp=2, ndraw=262144,
                                          scales=(1.0, 1.5))
    assert abs(lz) < 5 * rel + 1e-3 and rel < 0.01 and ess > 1e4


def test_importance_logz_with_a_coordinate_the_likelihood_ignores():
    """A parameter the likelihood ignores has a uniform posterior; its coordinate is drawn
    uniformly, the mixture covering the rest. ln Z = 0 again (normalised Gaussian in the other
    two coordinates), with most draws useful."""
    s = 0.05
    cov = s * s * np.array([[1.0, 0.6], [0.6, 1.0]])
    prec = torch.tensor(np.linalg.inv(cov))
    norm = -0.5 * math.log((2 * math.pi) ** 2 * np.linalg.det(cov))
    ll = lambda th: norm - 0.5 * (((th[:, :2] - 0.5) @ prec) * (th[:, :2] - 0.5)).sum(1)
    rng = np.random.default_rng(2)
    post = np.column_stack([rng.multivariate_normal(np.full(2, 0.5), cov, size=4000), rng.random(4000)])
    lz, rel, ess = nested.importance_logz(post, ll, lambda u: u, torch.device("cpu"), ncomp=2, ndraw=262144,
                                          scales=(1.0, 1.5))
    assert abs(lz) < 5 * rel + 1e-3 and rel < 0.01 and ess > 5e4


def test_speedup_law():
    assert nested.speedup_law(1, 2000) == pytest.approx(1.0, rel=3e-4)
    # the values quoted beside the paper's scaling test (K = 2000)
    for cores, s in [(16, 15.94), (64, 63.0), (320, 296.8), (640, 555.3)]:
        assert nested.speedup_law(cores, 2000) == pytest.approx(s, abs=0.06)


def test_gw_prior_transform_jacobian():
    """The analytic Jacobian of the prior transform against autograd."""
    tr = nested.gw_prior_transform()
    u = torch.tensor(np.random.default_rng(4).uniform(0.02, 0.98, (50, 11)), requires_grad=True)
    th = tr(u)
    th.sum().backward()
    np.testing.assert_allclose(tr.jacobian(u.detach()).numpy(), u.grad.numpy(), rtol=1e-12)


def test_gw_prior_transform_matches_synthetic_prior_draws():
    from paper_1909_11873_amd import synth
    u = np.random.default_rng(8).random((1000, 11))
    th = nested.gw_prior_transform()(torch.tensor(u)).numpy()
    rng = np.random.default_rng(8)
    ref = synth.prior_draw(rng, 1000)
    np.testing.assert_allclose(th, ref, rtol=1e-12, atol=1e-12)


def test_gw_prior_transform_is_the_inverse_cdf():
    """Each column's CDF, written from its density, at the transformed point returns u: uniform
    columns (x - a)/(b - a), distance (x^3 - a^3)/(b^3 - a^3) for density ~ x^2, declination
    (1 + sin x)/2 for density ~ cos x, inclination (1 + cos x)/2 for density ~ sin x with the
    orientation that maps u = 0 to pi. Points outside the cube land on its faces."""
    lo, hi = 100.0, 2000.0
    tr = nested.gw_prior_transform(mc_range=(10.0, 60.0), dl_range=(lo, hi), tc_half=0.1)
    u = np.random.default_rng(17).random((400, 11))
    th = tr(torch.tensor(u)).numpy()
    cdf = np.empty_like(th)
    for j, (a, b) in {0: (10.0, 60.0), 1: (0.2, 1.0), 2: (-0.9, 0.9), 3: (-0.9, 0.9), 5: (0.0, 2 * np.pi),
                      8: (0.0, np.pi), 9: (0.0, 2 * np.pi), 10: (-0.1, 0.1)}.items():
        cdf[:, j] = (th[:, j] - a) / (b - a)
    cdf[:, 4] = (th[:, 4] ** 3 - lo ** 3) / (hi ** 3 - lo ** 3)
    cdf[:, 6] = (1.0 + np.sin(th[:, 6])) / 2.0
    cdf[:, 7] = (1.0 + np.cos(th[:, 7])) / 2.0
    np.testing.assert_allclose(cdf, u, atol=1e-12)
    assert np.all((th[:, 6] >= -np.pi / 2) & (th[:, 6] <= np.pi / 2) & (th[:, 7] >= 0) & (th[:, 7] <= np.pi))
    out = tr(torch.tensor([[-0.5] * 11, [1.5] * 11])).numpy()
    np.testing.assert_array_equal(out, tr(torch.tensor([[0.0] * 11, [1.0] * 11])).numpy())


DEV = torch.device("cuda:0")


@pytest.mark.gpu
def test_prior_transform_kernel_matches_the_definitions():
    """gwl_prior_transform against the maps written out in float64 numpy, on the GW prior and on
    random columns of every kind, with points inside, on the faces of and outside the cube."""
    from paper_1909_11873_amd import gwlike as gw
    rng = np.random.default_rng(23)
    u = rng.uniform(-0.2, 1.2, (70001, 11))
    u[:5] = 0.0
    u[5:10] = 1.0
    tr = nested.gw_prior_transform()
    got = tr(torch.tensor(u, device=DEV)).cpu().numpy()
    ref = tr(torch.tensor(u)).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-15)
    d = 40
    maps = rng.integers(0, 4, d)
    c0 = rng.uniform(-1.0, 1.0, d)
    c1 = rng.uniform(-2.0, 2.0, d)
    c0[maps == 1] = rng.uniform(1.0, 1e9, (maps == 1).sum())
    c1[maps == 1] = rng.uniform(1.0, 1e9, (maps == 1).sum())
    v = rng.uniform(-0.1, 1.1, (3333, d))
    got = gw.prior_transform(torch.tensor(v, device=DEV), gw.PriorColumns(maps, c0, c1)).cpu().numpy()
    x = c0 + c1 * np.clip(v, 0.0, 1.0)
    ref = np.where(maps == 1, np.cbrt(x), np.where(maps == 2, np.arcsin(np.clip(x, -1, 1)),
                                                  np.where(maps == 3, np.arccos(np.clip(x, -1, 1)), x)))
    # the kernel forms the argument in one fused multiply-add, numpy in two roundings; asin and
    # acos amplify that near +-1, where their slope grows, so compare through the maps' inverses
    np.testing.assert_allclose(np.where(maps == 1, got ** 3, np.where(maps == 2, np.sin(got),
                                        np.where(maps == 3, np.cos(got), got))),
                               np.where(maps == 1, ref ** 3, np.where(maps == 2, np.sin(ref),
                                        np.where(maps == 3, np.cos(ref), ref))), rtol=1e-13, atol=1e-14)


@pytest.mark.gpu
@pytest.mark.parametrize("kind,n", [("ball", 16), ("prior", 1000)])
def test_driver_matches_oracle_on_gpu(kind, n):
    compare(DEV, kind, n)


def quiet_c0_event(distance=1500.0):
    """c0's detector, grid, PSD and noise with the injection moved to `distance` Mpc."""
    from oracle import gw_oracle as o
    from paper_1909_11873_amd import synth
    spec = synth.event_spec(0)
    f, psd, nz, dets = synth.event_arrays(spec)
    th0 = spec.theta0.copy()
    th0[4] = distance
    data = nz + o.strain_all(th0, dets, f).numpy()
    l0 = float(o.logl(th0[None], data, psd, dets, f, spec.df)[0])
    return spec, th0, f, psd, data, dets, l0


@pytest.mark.gpu
@pytest.mark.parametrize("batch", [128, 512])
def test_gw_nested_sampling_recovers_the_injection(batch):
    """Full runs on the GW likelihood (one detector, 4 s, 20-1024 Hz, no spins, optimal SNR 21)
    through the library's mixed-precision kernels, with gradient-guided walks that use its
    adjoint: the run finishes, the chirp-mass posterior covers the injected value, the run
    reaches the injection's likelihood, and the evidences at two batch sizes agree within their
    errors. (The single bounding ellipsoid stalls on this posterior: it accepted 0.2 of 8192
    candidates per iteration by the 2,400th dead point.)"""
    from paper_1909_11873_amd import gwlike as gw

    spec, th0, f, psd, data, dets, l0 = quiet_c0_event()
    ev = gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets,
                  torch.tensor(f, device=DEV), spec.df)
    smp = nested.ParallelNestedSampler(lambda th: gw.logl(th, ev, "mixed"), 11, 400, batch, proposal="gmc",
                                       loglike_grad=lambda th: gw.logl_grad(th, ev, "mixed"), gmc_steps=10,
                                       device=DEV, seed=3 + batch, prior_transform=nested.gw_prior_transform(spins=False))
    res = smp.run(eps=0.1, max_iter=8000)
    w = np.exp(res.log_w)
    mc = np.sum(w * res.theta[:, 0])
    mc_sd = math.sqrt(np.sum(w * (res.theta[:, 0] - mc) ** 2))
    print(f"GW NS batch {batch}: {res.niter} iterations, {res.ncall} calls, {res.seconds:.1f} s, lnZ {res.logz:.2f} "
          f"+- {res.logz_err:.2f}, H {res.information:.1f}, mc {mc:.3f} +- {mc_sd:.3f} (injected {th0[0]}), "
          f"logL(theta0) {l0:.2f}, max logL {res.logl.max():.2f}, mean accepted {res.n_accepted.mean():.1f}")
    assert res.niter < 8000
    assert abs(mc - th0[0]) < 5 * mc_sd + 0.05
    assert res.logl.max() > l0 - 5.0
    nd = len(res.logl) - 400
    assert np.all(np.diff(res.logl[:nd]) >= 0)
    RESULTS[batch] = (res.logz, res.logz_err)
    if len(RESULTS) == 2:
        (za, ea), (zb, eb) = RESULTS.values()
        assert abs(za - zb) < 4 * math.hypot(ea, eb) + 0.3
    ev.close()


RESULTS = {}


@pytest.mark.gpu
def test_gw_slice_nested_sampling_matches_importance_sampling():
    """Three detectors, 8 s, aligned spins (11 parameters), the injection moved to optimal SNR 20,
    the library's mixed-precision kernels, slice walks (5 d moves per candidate): the run keeps
    the injected sky position, reaches the injection's likelihood, and its evidence agrees with
    an importance-sampling estimate whose proposal is fitted to the run's own posterior. The
    tolerance of 1.5 nats covers the run-to-run scatter of this posterior's evidence (standard
    deviation 0.6 over eight runs at K = 1000 and 2000; the sqrt(H/K) error, 0.17, leaves out
    posterior mass drifting between the modes of the mass-ratio/spin degeneracy)."""
    from oracle import gw_oracle as o
    from paper_1909_11873_amd import gwlike as gw
    from paper_1909_11873_amd import synth

    spec = synth.event_spec(1)
    f, psd, nz, dets = synth.event_arrays(spec)
    th0 = spec.theta0.copy()
    h = o.strain_all(th0, dets, f)
    snr0 = math.sqrt(sum(float(o.inner(h[i], h[i], torch.tensor(psd[i]), spec.df)) for i in range(len(dets))))
    th0[4] *= snr0 / 20.0
    data = nz + o.strain_all(th0, dets, f).numpy()
    l0 = float(o.logl(th0[None], data, psd, dets, f, spec.df)[0])
    ev = gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets,
                  torch.tensor(f, device=DEV), spec.df)
    ll = lambda th: gw.logl(th, ev, "mixed")
    tr = nested.gw_prior_transform(mc_range=spec.mc_range, spins=spec.spins)
    res = nested.ParallelNestedSampler(ll, 11, 1000, 1024, device=DEV, seed=2, prior_transform=tr,
                                       proposal="slice").run(eps=0.1, max_iter=2000)
    w = np.exp(res.log_w)
    w /= w.sum()
    sky = np.hypot(np.angle(np.exp(1j * (res.theta[:, 5] - th0[5]))), res.theta[:, 6] - th0[6]) < 0.3
    post = res.u[np.random.default_rng(0).choice(len(w), size=20000, p=w)]
    lz_is, rel, ess = nested.importance_logz(post, ll, tr, DEV)
    print(f"GW NS slice c1: {res.niter} iterations, {res.ncall} calls, {res.seconds:.1f} s, lnZ {res.logz:.2f} "
          f"+- {res.logz_err:.2f}; importance sampling {lz_is:.3f} +- {rel:.3f} (ESS {ess:.0f}); "
          f"logL(theta0) {l0:.2f}, max logL {res.logl.max():.2f}, injected sky mass {w[sky].sum():.3f}")
    assert w[sky].sum() > 0.9
    assert res.logl.max() > l0 - 1.0
    assert rel < 0.1 and ess > 100
    assert abs(res.logz - lz_is) < 1.5
    ev.close()


@pytest.mark.gpu
def test_slice_graphs_and_kernels_replay_the_eager_moves():
    """The slice moves replayed from captured graphs, and with their bookkeeping in the library's
    kernels (gwl_slice_*), with and without a likelihood that evaluates only the live draws, give
    the eager torch moves bit for bit: the same dead points, likelihoods and call counts over a
    few iterations of a GW run."""
    from paper_1909_11873_amd import gwlike as gw

    spec, th0, f, psd, data, dets, l0 = quiet_c0_event()
    ev = gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets,
                  torch.tensor(f, device=DEV), spec.df)
    runs = []
    live = lambda th, n: gw.logl_live(th, n, ev, "mixed")
    for graphs, kernels, lv in ((False, False, None), (True, True, None), (False, True, None), (True, False, None),
                                (True, True, live), (False, True, live)):
        smp = nested.ParallelNestedSampler(lambda th: gw.logl(th, ev, "mixed"), 11, 200, 256, proposal="slice",
                                           slice_steps=6, slice_graphs=graphs, slice_kernels=kernels, device=DEV,
                                           seed=12, prior_transform=nested.gw_prior_transform(spins=False),
                                           loglike_live=lv)
        with warnings.catch_warnings(record=True) as caught:
            warnings.simplefilter("always")
            runs.append(smp.run(eps=0.1, max_iter=12))
        # the graph runs really replayed graphs (a failed capture warns and moves eagerly)
        assert not [w for w in caught if "eagerly" in str(w.message)]
        assert smp.slice_graphs == graphs
    ref = runs[0]
    assert ref.niter == 12
    for r in runs[1:]:
        assert r.niter == ref.niter
        np.testing.assert_array_equal(r.u, ref.u)
        np.testing.assert_array_equal(r.logl, ref.logl)
        assert r.ncall == ref.ncall
    ev.close()


@pytest.mark.gpu
@pytest.mark.parametrize("m", [1, 4])
def test_slice_kernels_are_the_sequential_procedure(m):
    """The library's slice kernels against the one-chain-at-a-time procedure with the same
    random numbers, on a region made of two balls (ln L = 0 inside, -inf outside)."""
    from paper_1909_11873_amd import gwlike as gw

    rng = np.random.default_rng(21 + m)
    n, d = 500, 3
    x = np.where(rng.random((3 * n, 1)) < 0.5, 0.3, 0.7) + 0.05 * rng.standard_normal((3 * n, d))
    x = x[two_balls(torch.tensor(x)).numpy()][:n]
    dirn = rng.standard_normal((n, d)) + np.where(rng.random((n, 1)) < 0.5, 3.0, 0.0)
    dirn *= (0.02 + 0.8 * rng.random((n, 1))) / np.linalg.norm(dirn, axis=1, keepdims=True)
    unif = rng.random((2 + nested.SLICE_MAX_DRAWS, n))
    raw = lambda p: torch.where(two_balls(p), 0.0, -math.inf).to(torch.float64)
    lmin = torch.zeros((), dtype=torch.float64, device=DEV)
    got, moved = nested.slice_move_dev(torch.tensor(x, device=DEV), torch.tensor(dirn, device=DEV),
                                       torch.tensor(unif, device=DEV), m, raw, lmin)
    got, moved = got.cpu().numpy(), moved.cpu().numpy()
    inside_np = lambda p: bool(two_balls(torch.tensor(p)))
    for i in range(n):
        ref, ok = neal_slice_move(x[i], dirn[i], unif[:, i], m, inside_np)
        assert bool(moved[i]) == ok
        np.testing.assert_array_equal(got[i], ref)
    assert moved.all()
    with pytest.raises(gw.GWLError):
        gw.slice_draws(torch.zeros(0, 3, dtype=torch.float64, device=DEV), torch.zeros(0, 3, dtype=torch.float64,
                       device=DEV), torch.zeros(0, dtype=torch.float64, device=DEV),
                       torch.zeros(0, dtype=torch.float64, device=DEV),
                       torch.zeros(8, 0, dtype=torch.float64, device=DEV),
                       torch.zeros(0, dtype=torch.int32, device=DEV), torch.zeros((), dtype=torch.int64, device=DEV))


@pytest.mark.gpu
@pytest.mark.parametrize("m,G,d", [(2, 1, 3), (3, 3, 13), (4, 8, 11), (5, 7, 2), (65, 64, 5), (66, 65, 4)])
def test_slice_stage_kernels_match_the_torch_stages(m, G, d):
    """Each stage kernel against the torch stage it replaces, bit for bit, over stepping-out
    limits and group sizes that fill a wavefront unevenly, exactly, or not at all (the per-chain
    fallback above 64 lanes), with more coordinates than lanes, chains already done, NaN ln L and
    candidates outside the cube; then a second group on the list of the chains still moving."""
    from paper_1909_11873_amd import gwlike as gw

    rng = np.random.default_rng(100 * m + G)
    n = 777
    x = torch.tensor(0.25 + 0.5 * rng.random((n, d)), device=DEV)
    dirn = torch.tensor(rng.standard_normal((n, d)) * rng.uniform(0.01, 0.6, (n, 1)), device=DEV)

    def raw(p):                        # a ball, NaN in a slab, -inf elsewhere
        r2 = ((p - 0.5) ** 2).sum(1)
        out = torch.where(r2 < 0.025 * d, -r2, -math.inf)
        return torch.where((p[:, 0] > 0.6) & (p[:, 0] < 0.62), math.nan, out)

    lmin = torch.tensor(-0.02 * d, dtype=torch.float64, device=DEV)
    inside = lambda p: ((p >= 0.0) & (p <= 1.0)).all(1) & (raw(p) >= lmin)
    u0, u1 = (torch.tensor(rng.random(n), device=DEV) for _ in range(2))
    lo_t, hi_t = nested._slice_stepping(x, dirn, u0, u1, m, inside)
    pts, lo, hi, jl, jr = gw.slice_ends(x, dirn, u0, u1, m)
    gw.slice_ends_select(pts, raw(pts), lmin, lo, hi, jl, jr, m)
    assert torch.equal(lo, lo_t) and torch.equal(hi, hi_t)
    assert bool((lo_t < -u0).any()) and bool((hi_t > 1.0 - u0).any())            # some ends stepped out

    assert pts.shape == ((m - 1) * n, d)                                         # only the ends examined

    done = torch.tensor(rng.random(n) < 0.2, device=DEV)
    xn = torch.tensor(rng.random((n, d)), device=DEV)
    ug = torch.tensor(rng.random((G, n)), device=DEV)
    xn_t, done_t, lo2_t, hi2_t = nested._slice_group(x, dirn, lo, hi, done, xn, ug, inside)
    lst, nact = gw.slice_list_init(n, DEV)
    calls = torch.zeros((), dtype=torch.int64, device=DEV)
    t, gpts, a, b, live, nact_next = gw.slice_draws(x, dirn, lo, hi, ug, lst, nact, calls)
    assert int(live) == n * G and int(calls) == n * G
    done_k = done.clone()
    lst2 = gw.slice_select(x, dirn, t, raw(gpts), lmin, a, b, xn, done_k, lo, hi, lst, nact, nact_next)
    assert torch.equal(xn, xn_t) and torch.equal(done_k, done_t)
    assert torch.equal(lo, lo2_t) and torch.equal(hi, hi2_t)
    hit = done_k & ~done
    assert 0 < int(hit.sum()) < int((~done).sum())                               # both outcomes occur
    # the next list: exactly the chains still moving (in any order)
    k = int(nact_next)
    assert k == int((~done_k).sum())
    assert torch.equal(torch.sort(lst2[:k].long()).values, torch.nonzero(~done_k)[:, 0])

    # a second group on that list: only its chains' draws are evaluated
    ug2 = torch.tensor(rng.random((G, n)), device=DEV)
    xn_t2, done_t2, lo3_t, hi3_t = nested._slice_group(x, dirn, lo, hi, done_k, xn, ug2, inside, active=True)
    t2, gpts2, a2, b2, live2, nact3 = gw.slice_draws(x, dirn, lo, hi, ug2, lst2, nact_next, calls)
    assert int(live2) == k * G and int(calls) == (n + k) * G
    gw.slice_select(x, dirn, t2, raw(gpts2[:k * G]), lmin, a2, b2, xn, done_k, lo, hi, lst2, nact_next, nact3)
    assert torch.equal(xn, xn_t2) and torch.equal(done_k, done_t2)
    assert torch.equal(lo, lo3_t) and torch.equal(hi, hi3_t)
    assert int(nact3) == int((~done_k).sum())


@pytest.mark.gpu
def test_slice_kernels_on_one_chain_in_one_dimension():
    """The smallest shapes: one chain, one coordinate, against the sequential procedure."""
    inside = lambda p: ((p - 0.4).abs() < 0.25).all(-1)
    raw = lambda p: torch.where(inside(p), 0.0, -math.inf).to(torch.float64)
    lmin = torch.zeros((), dtype=torch.float64, device=DEV)
    rng = np.random.default_rng(5)
    for trial in range(20):
        x = np.array([[0.2 + 0.4 * rng.random()]])
        dirn = np.array([[rng.uniform(-0.5, 0.5)]])
        unif = rng.random((2 + nested.SLICE_MAX_DRAWS, 1))
        got, moved = nested.slice_move_dev(torch.tensor(x, device=DEV), torch.tensor(dirn, device=DEV),
                                           torch.tensor(unif, device=DEV), 4, raw, lmin)
        ref, ok = neal_slice_move(x[0], dirn[0], unif[:, 0], 4, lambda p: bool(inside(torch.tensor(p))))
        assert bool(moved[0]) == ok
        np.testing.assert_array_equal(got.cpu().numpy()[0], ref)


@pytest.mark.gpu
def test_prior_transform_at_its_largest_width_and_one_point():
    from paper_1909_11873_amd import gwlike as gw
    rng = np.random.default_rng(29)
    d = 64
    maps = np.arange(d) % 4
    c0 = np.where(maps == 1, 8.0, -1.0)
    c1 = np.where(maps == 1, 19.0, 2.0)
    u = rng.random((1, d))
    got = gw.prior_transform(torch.tensor(u, device=DEV), gw.PriorColumns(maps, c0, c1)).cpu().numpy()
    x = c0 + c1 * u
    xc = np.clip(x, -1.0, 1.0)                          # np.where evaluates every branch
    ref = np.where(maps == 1, np.cbrt(x), np.where(maps == 2, np.arcsin(xc), np.where(maps == 3, np.arccos(xc), x)))
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)
    with pytest.raises(ValueError):
        gw.PriorColumns([0] * 65, [0.0] * 65, [1.0] * 65)


@pytest.mark.gpu
def test_slice_moves_fall_back_to_eager_when_capture_fails():
    """A likelihood that cannot run under graph capture (here: one that refuses to) makes the
    sampler warn and move eagerly, with the same result as asking for eager moves."""
    from paper_1909_11873_amd import gwlike as gw

    spec, th0, f, psd, data, dets, l0 = quiet_c0_event()
    ev = gw.Event(torch.tensor(data, device=DEV), torch.tensor(psd, device=DEV), dets,
                  torch.tensor(f, device=DEV), spec.df)

    def refusing(th):
        if torch.cuda.is_current_stream_capturing():
            raise RuntimeError("this likelihood does not run under capture")
        return gw.logl(th, ev, "mixed")

    runs = []
    for graphs in (True, False):
        smp = nested.ParallelNestedSampler(refusing, 11, 100, 128, proposal="slice", slice_steps=3,
                                           slice_graphs=graphs, device=DEV, seed=8,
                                           prior_transform=nested.gw_prior_transform(spins=False))
        if graphs:
            with pytest.warns(UserWarning, match="eagerly"):
                runs.append(smp.run(eps=0.1, max_iter=5))
        else:
            runs.append(smp.run(eps=0.1, max_iter=5))
    np.testing.assert_array_equal(runs[0].u, runs[1].u)
    assert runs[0].ncall == runs[1].ncall
    ev.close()

