"""Static parallel nested sampling on one GPU, driving the batched likelihood.

This is the paper's section 3 ("Parallel Nested Sampling") and its algorithm "Static Parallel
Nested Sampling" with the pool of workers replaced by one batch of candidates per iteration.
Everything stays on the device; one iteration is a fixed sequence of launches with no host
synchronisation (the host reads the stop flag every few iterations; the slice-sampling proposal
also asks, after each group of shrinkage draws, whether every chain has finished):

  1. L_min is the first live log-likelihood (the live set is kept sorted ascending).
  2. n candidates in the unit cube: prior draws (the paper's proposal), draws from the bounding
     ellipsoid of the live points (the "bounding distribution" the algorithm re-evaluates each
     iteration), gradient-guided walks inside the current contour (Galilean Monte Carlo: straight
     steps from live points, reflected off the contour along the likelihood gradient, which the
     library's adjoint provides for a whole batch at once), slice-sampling walks inside the
     contour (random directions in the live points' whitened coordinates, stepping out and
     shrinkage; every chain moves, whatever the local scale), or a caller's proposal function.
  3. Prior transform and ln L of the whole batch (for the GW likelihood: the library's kernels).
  4. Candidates in the cube with L >= L_min are accepted (n' of them).
  5. The paper replaces the worst live point by each accepted candidate in turn. Taken in
     ascending order of L, that sequence removes exactly the n' lowest of the K + n' points
     (live and accepted): every candidate is then at or above the point it replaces, so the
     removed points come out in ascending order. One stable sort of the merged set therefore
     does the whole replacement loop: rejected candidates first, then the n' dead points in
     ascending L, then the K new live points.
  6. Prior volume: the first dead point of the iteration shrinks X by the largest of K uniform
     draws (ln X -= 1/K), the j-th (j >= 2) by the largest of K + n' - j + 1; this is the paper's
     ln X_i = -i/K when n' = 1. Evidence by the Riemann sum of dX_i L_i.
  7. Stop when the remaining volume can change ln Z by at most eps: ln(Z + L_max X) - ln Z <= eps.

At the end the K live points join the dead ones with equal shares of the last volume, and the
posterior weights are p_i = L_i dX_i / Z.
"""
from __future__ import annotations

import dataclasses
import math
import time
import warnings
from typing import Callable, Optional

import numpy as np
import torch


@dataclasses.dataclass
class NSResult:
    u: np.ndarray            # [N, d] dead points (then the final live points) in the unit cube
    theta: np.ndarray        # [N, d] the same points after the prior transform
    logl: np.ndarray         # [N]
    log_dx: np.ndarray       # [N] ln of each point's prior-volume share
    log_x: np.ndarray        # [N] ln X after each dead point (final live points: the shares left)
    logz: float
    logz_err: float          # sqrt(H / K)
    log_w: np.ndarray        # [N] ln posterior weight
    information: float       # H in nats
    niter: int
    ncall: int
    n_accepted: np.ndarray   # [niter] accepted candidates per iteration
    seconds: float

    def speedup(self) -> float:
        """Serial iterations the run replaced: K ln(1/X_end) / iterations (the measured S)."""
        nd = len(self.logl) - self.nlive
        return -self.log_x[nd - 1] * self.nlive / max(self.niter, 1) if nd > 0 else 0.0

    nlive: int = 0


def speedup_law(n: float, nlive: float) -> float:
    """The paper's speed-up relation S(n, K) = K ln(1 + n/K)."""
    return nlive * math.log1p(n / nlive)


def gw_prior_transform(mc_range=(10.0, 60.0), dl_range=(100.0, 2000.0), tc_half=0.1, spins=True):
    """Unit cube -> the 11 parameters (mc, q, chi1, chi2, dl, ra, dec, iota, psi, phic, tc) by the
    inverse CDFs of the prior: uniform mc, q in [0.2, 1], spins in [-0.9, 0.9], distance with
    density ~ d^2, isotropic sky and orientation, uniform angles and coalescence time. Each column
    is g(c0 + c1 u) with g the identity, the cube root (distance), asin (declination) or acos
    (inclination); points outside the cube are clamped into it first. On a CUDA tensor the
    library's gwl_prior_transform does the whole map in one launch."""
    lo3, hi3 = dl_range[0] ** 3, dl_range[1] ** 3
    sw = 1.8 if spins else 0.0
    c0 = [mc_range[0], 0.2, -sw / 2, -sw / 2, lo3, 0.0, -1.0, -1.0, 0.0, 0.0, -tc_half]
    c1 = [mc_range[1] - mc_range[0], 0.8, sw, sw, hi3 - lo3, 2.0 * math.pi, 2.0, 2.0, math.pi, 2.0 * math.pi,
          2.0 * tc_half]
    maps = [0, 0, 0, 0, 1, 0, 2, 3, 0, 0, 0]       # identity, cube root (4), asin (6), acos (7)
    consts = {}

    def transform(u: torch.Tensor) -> torch.Tensor:
        if u.is_cuda and u.dtype == torch.float64 and not u.requires_grad:
            from . import gwlike as gw
            if "cols" not in consts:
                consts["cols"] = gw.PriorColumns(maps, c0, c1)
            return gw.prior_transform(u, consts["cols"])
        key = (u.device, u.dtype)
        if key not in consts:
            consts[key] = (torch.tensor(c0, device=u.device, dtype=u.dtype),
                           torch.tensor(c1, device=u.device, dtype=u.dtype))
        a, b = consts[key]
        x = torch.addcmul(a, u.clamp(0.0, 1.0), b)
        th = x.clone()
        th[:, 4] = torch.pow(x[:, 4], 1.0 / 3.0)
        s67 = x[:, 6:8].clamp(-1.0, 1.0)
        th[:, 6] = torch.asin(s67[:, 0])
        th[:, 7] = torch.acos(s67[:, 1])
        return th

    def jacobian(u: torch.Tensor) -> torch.Tensor:
        """d theta_i / d u_i (the transform acts column by column)."""
        j = torch.empty_like(u)
        j[:, 0] = mc_range[1] - mc_range[0]
        j[:, 1] = 0.8
        j[:, 2:4] = 1.8 if spins else 0.0
        j[:, 4] = (hi3 - lo3) / 3.0 * torch.pow(lo3 + u[:, 4] * (hi3 - lo3), -2.0 / 3.0)
        j[:, 5] = 2.0 * math.pi
        s6 = 1.0 - (2.0 * u[:, 6] - 1.0) ** 2
        s7 = 1.0 - (2.0 * u[:, 7] - 1.0) ** 2
        j[:, 6] = 2.0 / torch.sqrt(s6.clamp(min=1e-300))
        j[:, 7] = -2.0 / torch.sqrt(s7.clamp(min=1e-300))
        j[:, 8] = math.pi
        j[:, 9] = 2.0 * math.pi
        j[:, 10] = 2.0 * tc_half
        return j

    transform.jacobian = jacobian
    transform.clamps = True
    return transform


SLICE_GROUPS = (8, 8, 16, 16)     # shrinkage draws evaluated together, group by group
SLICE_MAX_DRAWS = sum(SLICE_GROUPS)   # draws per slice move before a chain gives up that move
SLICE_GROUP = SLICE_GROUPS[0]


def _slice_groups():
    """(first row of unif, group size) of every shrinkage group of a move."""
    off = 2
    for g in SLICE_GROUPS:
        yield off, g
        off += g


def slice_move(x, dirn, unif, m, inside):
    """One slice-sampling move per chain for the uniform distribution on a region (stepping out
    and shrinkage along a line, Neal 2003, sections 4.1 and 4.2).

    x[n, d]: the chains' points (inside the region); dirn[n, d]: each chain's direction, whose
    length is the initial interval's; unif[2 + SLICE_MAX_DRAWS, n]: uniform numbers, row 0 the
    interval's offset, row 1 the split of the m - 1 stepping-out steps between the two ends, the
    rest the shrinkage draws in order; inside(p[N, d]) -> bool[N].
    Returns (new points, whether each chain moved).

    The interval [x - r dirn, x + (1 - r) dirn] steps out by whole lengths, at most J times to
    the left and m - 1 - J times to the right (J = floor(m v)), while its end lies inside; then
    draws uniformly from it, shrinking it to the draw after every draw outside, until a draw
    lands inside. The line need not cross the region in one piece: the move leaves the uniform
    distribution on the region invariant all the same, and never returns its start point.

    The outcome is fixed by the uniform numbers and by which of the points the procedure looks at
    lie inside, so those points are evaluated ahead, in one batch per stage: the m - 1 ends the
    stepping out can examine (J on the left, m - 1 - J on the right), then the shrinkage draws in
    groups (SLICE_GROUPS) for the chains still moving, each draw from the interval as it would be
    if the earlier draws of its group had fallen outside. The first draw inside is the one the
    sequential procedure returns. A chain with no draw inside after SLICE_MAX_DRAWS keeps its
    point."""
    lo, hi = _slice_stepping(x, dirn, unif[0], unif[1], m, inside)
    done = torch.zeros(x.shape[0], dtype=torch.bool, device=x.device)
    xn = x
    for r0, G in _slice_groups():
        xn, done, lo, hi = _slice_group(x, dirn, lo, hi, done, xn, unif[r0:r0 + G], inside)
        if bool(done.all()):
            break
    return xn, done


def _slice_stepping(x, dirn, u0, u1, m, inside):
    """The interval of a slice move after stepping out: (lo, hi) in units of dirn. Slot s of a
    chain is its left end lo - s for s < J and its right end hi + (s - J) from there on."""
    n, d = x.shape
    lo, hi = -u0, 1.0 - u0
    if m > 1:
        jl = torch.floor(m * u1)
        jr = (m - 1) - jl
        s = torch.arange(m - 1, dtype=x.dtype, device=x.device)[:, None]                    # [m - 1, 1]
        left = s < jl[None]                                                                  # [m - 1, n]
        t = torch.where(left, lo[None] - s, hi[None] + (s - jl[None]))
        ok = inside((x[None] + t[..., None] * dirn[None]).reshape(-1, d)).reshape(m - 1, n)
        out_l, out_r = left & ~ok, ~left & ~ok
        sl = torch.where(out_l.any(0), torch.argmax(out_l.to(torch.int8), 0).to(x.dtype), jl)
        sr = torch.where(out_r.any(0), torch.argmax(out_r.to(torch.int8), 0).to(x.dtype) - jl, jr)
        lo = lo - sl
        hi = hi + sr
    return lo, hi


def _slice_group(x, dirn, lo, hi, done, xn, ug, inside, active=False):
    """One group of shrinkage draws (ug[G, n], in order) for the chains not done yet. With
    active=True only those chains' draws are passed to inside() (a host synchronisation);
    otherwise every chain's draws are, and the done ones ignored."""
    n, d = x.shape
    ts = []
    a, b = lo, hi
    for k in range(ug.shape[0]):
        t = a + ug[k] * (b - a)
        ts.append(t)
        left = t < 0.0
        a, b = torch.where(left, t, a), torch.where(left, b, t)
    tt = torch.stack(ts)                                                                  # [G, n]
    if active:
        act = torch.nonzero(~done)[:, 0]
        ok = torch.zeros(ug.shape[0], n, dtype=torch.bool, device=x.device)
        if act.numel():
            pa = (x[act][None] + tt[:, act, None] * dirn[act][None]).reshape(-1, d)
            ok[:, act] = inside(pa).reshape(ug.shape[0], -1)
    else:
        ok = inside((x[None] + tt[..., None] * dirn[None]).reshape(-1, d)).reshape(ug.shape[0], n)
    ok = ok & ~done[None]
    hit = ok.any(0)
    tsel = tt.gather(0, torch.argmax(ok.to(torch.int8), 0)[None])[0]
    xn = torch.where(hit[:, None], x + tsel[:, None] * dirn, xn)
    done = done | hit
    return xn, done, torch.where(done, lo, a), torch.where(done, hi, b)


def _slice_stepping_dev(x, dirn, u0, u1, m, raw, lmin):
    """_slice_stepping with the library's kernels (gwl_slice_ends / _ends_select); raw(p) is
    ln L at the points p (NaN allowed), lmin a device scalar. Same arithmetic, same results."""
    if m <= 1:
        return -u0, 1.0 - u0
    from . import gwlike as gw
    pts, lo, hi, jl, jr = gw.slice_ends(x, dirn, u0, u1, m)
    gw.slice_ends_select(pts, raw(pts), lmin, lo, hi, jl, jr, m)
    return lo, hi


def _slice_group_dev(x, dirn, lo, hi, done, xn, ug, live_eval, lmin, lst, nact, calls=None):
    """_slice_group with the library's kernels (gwl_slice_draws / _select) for the listed chains,
    in place on xn, done, lo and hi; live_eval(pts, live) is ln L at the first `live` rows of pts
    (live a device int64 scalar). Returns the next list and its length (device)."""
    from . import gwlike as gw
    t, pts, a, b, live, nact_next = gw.slice_draws(x, dirn, lo, hi, ug, lst, nact, calls)
    logl = live_eval(pts, live)
    lst_next = gw.slice_select(x, dirn, t, logl, lmin, a, b, xn, done, lo, hi, lst, nact, nact_next)
    return lst_next, nact_next


def _eager_live(raw):
    """live_eval for eager moves: reads the live count (a host synchronisation) and evaluates
    exactly those rows."""
    def live_eval(pts, live):
        k = int(live)
        return raw(pts[:k]) if k else torch.empty(0, dtype=torch.float64, device=pts.device)
    return live_eval


def slice_move_dev(x, dirn, unif, m, raw, lmin, calls=None):
    """slice_move with the bookkeeping in the library's kernels: the candidate ends and draws
    are written by one kernel per stage and judged by another, between them one call of raw(p)
    (ln L at the points, NaN allowed); the region is {p in the cube, ln L(p) >= lmin}. Shrinkage
    groups evaluate only the chains still moving; `calls` (a device int64, optional) counts their
    draws."""
    from . import gwlike as gw
    lo, hi = _slice_stepping_dev(x, dirn, unif[0], unif[1], m, raw, lmin)
    lo, hi = lo.contiguous(), hi.contiguous()
    done = torch.empty(x.shape[0], dtype=torch.bool, device=x.device)
    xn = torch.empty_like(x)
    lst, nact = gw.slice_move_begin(x, xn, done)
    live_eval = _eager_live(raw)
    for r0, G in _slice_groups():
        lst, nact = _slice_group_dev(x, dirn, lo, hi, done, xn, unif[r0:r0 + G], live_eval, lmin, lst, nact, calls)
        if int(nact) == 0:
            break
    return xn, done


class _SliceGraphs:
    """The slice moves of one batch shape captured as one HIP graph per move: the move's
    direction, stepping out, and all its groups of shrinkage draws (SLICE_GROUPS), each
    group for the chains still moving (a list kept on the device, so a group after every chain is
    done costs only its empty launches and no host decision is needed). The host draws each move's
    random numbers into static buffers (the same calls, in the same order, as the eager path, so
    both paths give the same chains bit for bit) and replays the graph; the likelihood calls
    inside (prior transform, the library's kernels) are part of the graph, with the device
    addresses they had at capture: the sampler captures again at the start of every run, and the
    likelihood's data (an event's tables) must stay alive while a run lasts. The draws evaluated
    are counted on the device (calls)."""

    def __init__(self, smp):
        n, d, m = smp.n, smp.d, smp.slice_out
        f64 = dict(dtype=torch.float64, device=smp.dev)
        self.smp = smp
        # placeholders for the warm-up and the capture: points at the cube's centre, unit directions
        self.x, self.z, self.dirn, self.xn = (torch.full((n, d), 0.5, **f64) for _ in range(4))
        self.unif = torch.full((2 + SLICE_MAX_DRAWS, n), 0.5, **f64)
        self.chol = torch.eye(d, **f64)
        self.lmin = torch.full((), -math.inf, **f64)
        self.done = torch.zeros(n, dtype=torch.bool, device=smp.dev)
        self.moved = torch.zeros(n, dtype=torch.bool, device=smp.dev)
        self.calls = torch.zeros((), dtype=torch.int64, device=smp.dev)
        stepping, group, begin, _, end = smp._slice_stages(self.lmin, count=False, calls=self.calls)

        def move():
            self.dirn.copy_(smp.slice_width * (self.z / self.z.norm(dim=1, keepdim=True)) @ self.chol.T)
            lo, hi = stepping(self.x, self.dirn, self.unif[0], self.unif[1])
            lo, hi = lo.contiguous(), hi.contiguous()
            state = begin(self.x, self.xn, self.done)
            for r0, G in _slice_groups():
                state = group(self.x, self.dirn, lo, hi, self.done, self.xn, self.unif[r0:r0 + G], state)
            end(self.done, self.moved, self.xn, self.x)

        side = torch.cuda.Stream(device=smp.dev)
        side.wait_stream(torch.cuda.current_stream(smp.dev))
        with torch.cuda.stream(side):            # warm-up outside capture (allocator, kernels)
            move()
        torch.cuda.current_stream(smp.dev).wait_stream(side)
        torch.cuda.synchronize(smp.dev)
        # captured on the warm-up's stream: the library keeps its workspace per stream and grows it
        # only outside capture, so the warm-up has reserved what the captured calls use
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=side):
            move()
        self.calls.zero_()
        self.calls_step = (m - 1) * n if m > 1 else 0       # stepping-out ends per move

    def walk(self, x0, chol, lmin, steps):
        """(points, whether each chain moved at least once)."""
        smp, n, d = self.smp, self.smp.n, self.smp.d
        self.x.copy_(x0)
        self.chol.copy_(chol)
        self.lmin.copy_(lmin)
        self.moved.zero_()
        for _ in range(steps):
            torch.randn(n, d, generator=smp.gen, out=self.z)
            torch.rand(2 + SLICE_MAX_DRAWS, n, generator=smp.gen, out=self.unif)
            self.graph.replay()
            smp.extra_calls += self.calls_step
        return self.x.clone(), self.moved.clone()


class ParallelNestedSampler:
    """K live points, n candidates per iteration, everything on `device`.

    loglike(theta[n, d]) -> ln L[n] (float64 tensors on the device; NaN counts as -inf).
    prior_transform(u[n, d]) -> theta[n, d]; identity if None.
    proposal: "prior", "ellipsoid", "gmc", "slice", or a function (it, live_u, live_l) -> u[n, d].
    loglike_grad(theta[n, d]) -> (ln L[n], d ln L / d theta [n, d]): needed for "gmc".
    slice_steps, slice_width, slice_out: slice moves per candidate, the initial interval length in
    units of the live points' spread along the direction, and the stepping-out limit m.
    loglike_live(theta[N, d], live) -> ln L[N] evaluated on the first `live` rows only (live a
    device int64 scalar, e.g. the library's logl_live): lets captured slice moves evaluate only
    the draws of the chains still moving. Without it they evaluate every row.
    """

    def __init__(self, loglike: Callable, ndim: int, nlive: int, batch: int,
                 prior_transform: Optional[Callable] = None, device="cuda:0", seed: int = 0,
                 proposal="ellipsoid", enlarge: float = 1.25, volume: str = "order", check_every: int = 8,
                 loglike_grad: Optional[Callable] = None, gmc_steps: int = 20, slice_steps: Optional[int] = None,
                 slice_width: float = 3.0, slice_out: int = 4, slice_graphs: bool = True,
                 slice_kernels: Optional[bool] = None, loglike_live: Optional[Callable] = None):
        if nlive < 2 or batch < 1 or ndim < 1:
            raise ValueError("need nlive >= 2, batch >= 1, ndim >= 1")
        if volume not in ("order", "paper"):
            raise ValueError("volume is 'order' or 'paper'")
        self.loglike, self.d, self.K, self.n = loglike, ndim, nlive, batch
        self.transform = prior_transform if prior_transform is not None else (lambda u: u)
        self.dev = torch.device(device)
        self.gen = torch.Generator(device=self.dev)
        self.gen.manual_seed(seed)
        self.proposal, self.enlarge, self.volume = proposal, enlarge, volume
        self.check_every = max(1, int(check_every))
        if proposal == "gmc" and loglike_grad is None:
            raise ValueError("proposal 'gmc' needs loglike_grad")
        self.loglike_grad, self.gmc_steps = loglike_grad, max(1, int(gmc_steps))
        self.gmc_scale = 0.5            # step length in units of the live points' spread, adapted
        self.slice_steps = max(1, int(slice_steps)) if slice_steps is not None else 5 * ndim
        if slice_width <= 0.0 or slice_out < 1:
            raise ValueError("need slice_width > 0 and slice_out >= 1")
        self.slice_width, self.slice_out = float(slice_width), int(slice_out)
        # slice moves replayed from captured graphs on a CUDA device (None: not built yet)
        self.slice_graphs_requested = bool(slice_graphs) and self.dev.type == "cuda"
        # slice-move bookkeeping in the library's kernels (default on a CUDA device), else in
        # torch array operations; both give the same chains
        self.slice_kernels = (self.dev.type == "cuda") if slice_kernels is None else bool(slice_kernels)
        if self.slice_kernels and self.dev.type != "cuda":
            raise ValueError("slice_kernels needs a CUDA device")
        self.slice_graphs = self.slice_graphs_requested
        self._graphs = None
        self.loglike_live = loglike_live
        self.extra_calls = 0
        # shrinkage draws evaluated, counted on the device (read once at the end of a run)
        self._calls_dev = torch.zeros((), dtype=torch.int64, device=self.dev)

    # ---- proposals -------------------------------------------------------------------------
    def _prior(self):
        return torch.rand(self.n, self.d, generator=self.gen, device=self.dev, dtype=torch.float64)

    def _ellipsoid(self, live_u):
        """Uniform draws in the bounding ellipsoid of the live points, its volume enlarged."""
        d = self.d
        mu = live_u.mean(0)
        x = live_u - mu
        cov = x.T @ x / (self.K - 1) + 1e-12 * torch.eye(d, dtype=torch.float64, device=self.dev)
        chol, _ = torch.linalg.cholesky_ex(cov)
        y = torch.linalg.solve_triangular(chol, x.T, upper=False)           # [d, K]
        r2 = (y * y).sum(0).max()                                            # all live points inside
        scale = torch.sqrt(r2) * self.enlarge ** (1.0 / d)
        z = torch.randn(self.n, d, generator=self.gen, device=self.dev, dtype=torch.float64)
        z = z / z.norm(dim=1, keepdim=True)
        rad = torch.rand(self.n, 1, generator=self.gen, device=self.dev, dtype=torch.float64) ** (1.0 / d)
        return mu + scale * (z * rad) @ chol.T

    def _grad_u(self, u):
        """ln L and its gradient in the unit cube (chain rule through the prior transform)."""
        jac = getattr(self.transform, "jacobian", None)
        if jac is not None:
            l, g = self.loglike_grad(self.transform(u))
            gu = g * jac(u)
            l = torch.where(torch.isnan(l), torch.full_like(l, -math.inf), l)
            return l, torch.where(torch.isfinite(gu), gu, torch.zeros_like(gu))
        uu = u.detach().clone().requires_grad_(True)
        with torch.enable_grad():
            th = self.transform(uu)
            l, g = self.loglike_grad(th.detach())
            th.backward(g)
        gu = uu.grad
        l = torch.where(torch.isnan(l), torch.full_like(l, -math.inf), l)
        gu = torch.where(torch.isfinite(gu), gu, torch.zeros_like(gu))
        return l.detach(), gu

    @staticmethod
    def _reflect_cube(x, v):
        """Mirror positions (and the velocity components) that left the unit cube."""
        lo, hi = x < 0.0, x > 1.0
        x = torch.where(lo, -x, torch.where(hi, 2.0 - x, x))
        v = torch.where(lo | hi, -v, v)
        return x.clamp(0.0, 1.0), v

    def _gmc(self, live_u, live_l):
        """Galilean Monte Carlo inside the contour L >= L_min, one chain per candidate, in the
        coordinates that whiten the live points (y = L^-1 (u - mean), C = L L^T their covariance;
        the uniform prior stays uniform under this affine map).

        Each chain starts at a random live point with a random isotropic velocity of length
        gmc_scale in y. A step moves straight ahead; if the new point is below L_min the velocity
        is reflected off the contour, v_y -> v_y - 2 (v_y.n) n with n the unit gradient of ln L in
        y (in u: v -> v - 2 (v.g) / (g^T C g) C g, g the gradient in u), and the step is retried
        from that point; if that also fails the velocity reverses. The cube's faces mirror the
        position. Chains that never moved are returned outside the cube (rejected), so no live
        point is duplicated."""
        n, d = self.n, self.d
        lmin = live_l[0]
        start = torch.randint(0, self.K, (n,), generator=self.gen, device=self.dev)
        x = live_u[start]
        xc = live_u - live_u.mean(0)
        cov = xc.T @ xc / (self.K - 1) + 1e-14 * torch.eye(d, dtype=torch.float64, device=self.dev)
        chol, _ = torch.linalg.cholesky_ex(cov)
        z = torch.randn(n, d, generator=self.gen, device=self.dev, dtype=torch.float64)
        v = self.gmc_scale * (z / z.norm(dim=1, keepdim=True)) @ chol.T
        moved = torch.zeros(n, dtype=torch.bool, device=self.dev)
        acc_moves = torch.zeros((), dtype=torch.float64, device=self.dev)
        for _ in range(self.gmc_steps):
            x1, v1 = self._reflect_cube(x + v, v)
            l1, g1 = self._grad_u(x1)
            ok1 = l1 >= lmin
            cg = g1 @ cov
            gcg = (g1 * cg).sum(1, keepdim=True).clamp(min=1e-300)
            vr = v1 - 2.0 * (v1 * g1).sum(1, keepdim=True) / gcg * cg
            x2, vr = self._reflect_cube(x1 + vr, vr)
            l2, _ = self._loglike(x2)
            ok2 = ~ok1 & (l2 >= lmin)
            x = torch.where(ok1[:, None], x1, torch.where(ok2[:, None], x2, x))
            v = torch.where(ok1[:, None], v1, torch.where(ok2[:, None], vr, -v))
            moved = moved | ok1 | ok2
            acc_moves = acc_moves + ok1.to(torch.float64).mean()
        self.extra_calls += 2 * n * self.gmc_steps
        # fraction of straight steps that stayed inside the contour; the host reads it at its
        # sync points and adapts the step length towards one half
        self._gmc_rate = acc_moves / self.gmc_steps
        return torch.where(moved[:, None], x, torch.full_like(x, 2.0))

    def _inside_raw(self, u, lmin):
        l, inside = self._loglike(u)
        return inside & (l >= lmin)

    def _in_contour(self, u, lmin):
        self.extra_calls += u.shape[0]
        return self._inside_raw(u, lmin)

    def _raw(self, u):
        """ln L at the points u (clamped into the cube), NaN kept: the slice kernels judge the
        cube and the contour themselves."""
        if getattr(self.transform, "clamps", False):
            return self.loglike(self.transform(u))
        return self.loglike(self.transform(u.clamp(0.0, 1.0)))

    def _slice_stages(self, lmin, count=True, calls=None):
        """(stepping(x, dirn, u0, u1) -> (lo, hi), group(x, dirn, lo, hi, done, xn, ug, state) ->
        state, begin(x, xn, done) -> state (xn = x, done = False), finished(state, done) -> bool,
        end(done, moved, xn, x) (moved |= done, x = xn)) for the contour ln L >= lmin, in the
        library's kernels or in torch. group updates xn, done, lo and hi in place and counts
        the draws it evaluates (those of the chains still moving) into `calls` (a device int64,
        the sampler's own if None); with count=True the stepping-out ends are counted on the host.
        With count=False (graph capture) nothing waits for the device."""
        m = self.slice_out
        calls = self._calls_dev if calls is None else calls

        def raw(p):
            if count:
                self.extra_calls += p.shape[0]
            return self._raw(p)
        if self.slice_kernels:
            from . import gwlike as gw
            # eager and captured moves evaluate the same rows with the same launches, so their
            # likelihood values agree bit for bit
            live_eval = self._raw_live

            def group(x, dirn, lo, hi, done, xn, ug, state):
                return _slice_group_dev(x, dirn, lo, hi, done, xn, ug, live_eval, lmin, state[0], state[1], calls)
            return (lambda x, dirn, u0, u1: _slice_stepping_dev(x, dirn, u0, u1, m, raw, lmin), group,
                    gw.slice_move_begin, lambda state, done: int(state[1]) == 0, gw.slice_move_end)
        inside = lambda p: self._inside_raw(p, lmin)
        inside_count = (lambda p: self._in_contour(p, lmin)) if count else inside

        def group(x, dirn, lo, hi, done, xn, ug, state):
            calls.add_(ug.shape[0] * (~done).sum())
            xn2, done2, lo2, hi2 = _slice_group(x, dirn, lo, hi, done, xn, ug, inside, active=count)
            for dst, src in ((xn, xn2), (done, done2), (lo, lo2), (hi, hi2)):
                if dst is not src:
                    dst.copy_(src)
            return state

        def begin(x, xn, done):
            done.zero_()
            xn.copy_(x)

        def end(done, moved, xn, x):
            moved |= done
            x.copy_(xn)
        return (lambda x, dirn, u0, u1: _slice_stepping(x, dirn, u0, u1, m, inside_count), group,
                begin, lambda state, done: bool(done.all()), end)

    def _raw_live(self, p, live):
        """ln L at the first `live` rows of p (a device int64 scalar) when the sampler has a
        loglike_live, else at every row."""
        th = self.transform(p) if getattr(self.transform, "clamps", False) else self.transform(p.clamp(0.0, 1.0))
        if self.loglike_live is not None:
            return self.loglike_live(th, live)
        return self.loglike(th)

    def _slice(self, live_u, live_l):
        """Slice-sampling walks inside the contour L >= L_min, one chain per candidate: each chain
        starts at a random live point and makes slice_steps moves of `slice_move`, along random
        directions isotropic in the coordinates that whiten the live points, each of length
        slice_width in those coordinates. A chain whose every move gave up (no shrinkage draw
        inside) is still at its live point: it is returned outside the cube, so it is rejected
        instead of duplicating that point."""
        n, d, K = self.n, self.d, self.K
        f64 = dict(dtype=torch.float64, device=self.dev)
        lmin = live_l[0]
        start = torch.randint(0, K, (n,), generator=self.gen, device=self.dev)
        x = live_u[start].clone()
        xc = live_u - live_u.mean(0)
        cov = xc.T @ xc / (K - 1) + 1e-14 * torch.eye(d, **f64)
        chol, _ = torch.linalg.cholesky_ex(cov)
        if self.slice_graphs and self._graphs is None:
            try:
                self._graphs = _SliceGraphs(self)
            except Exception as exc:      # a likelihood that cannot be captured: eager moves
                warnings.warn(f"slice moves run eagerly: capturing them failed ({exc})")
                self.slice_graphs = False
                self._graphs = None
        if self.slice_graphs:
            x, moved = self._graphs.walk(x, chol, lmin, self.slice_steps)
            return torch.where(moved[:, None], x, torch.full_like(x, 2.0))
        stepping, group, begin, finished, end = self._slice_stages(lmin)
        moved = torch.zeros(n, dtype=torch.bool, device=self.dev)
        done = torch.empty(n, dtype=torch.bool, device=self.dev)
        xn = torch.empty_like(x)
        for _ in range(self.slice_steps):
            z = torch.randn(n, d, generator=self.gen, **f64)
            dirn = self.slice_width * (z / z.norm(dim=1, keepdim=True)) @ chol.T
            unif = torch.rand(2 + SLICE_MAX_DRAWS, n, generator=self.gen, **f64)
            lo, hi = stepping(x, dirn, unif[0], unif[1])
            lo, hi = lo.contiguous(), hi.contiguous()
            state = begin(x, xn, done)
            for r0, G in _slice_groups():
                state = group(x, dirn, lo, hi, done, xn, unif[r0:r0 + G], state)
                if finished(state, done):
                    break
            end(done, moved, xn, x)
        return torch.where(moved[:, None], x, torch.full_like(x, 2.0))

    def _propose(self, it, live_u, live_l):
        if callable(self.proposal):
            return self.proposal(it, live_u, live_l)
        if self.proposal == "prior":
            return self._prior()
        if self.proposal == "ellipsoid":
            return self._ellipsoid(live_u)
        if self.proposal == "gmc":
            return self._gmc(live_u, live_l)
        if self.proposal == "slice":
            return self._slice(live_u, live_l)
        raise ValueError(f"unknown proposal {self.proposal!r}")

    def _loglike(self, u):
        inside = ((u >= 0.0) & (u <= 1.0)).all(dim=1)
        l = self.loglike(self.transform(u.clamp(0.0, 1.0)))
        l = torch.where(torch.isnan(l), torch.full_like(l, -math.inf), l)
        return l, inside

    # ---- the run ---------------------------------------------------------------------------
    def run(self, eps: float = 0.1, max_iter: int = 100000, live_u: Optional[torch.Tensor] = None) -> NSResult:
        K, n, d, dev = self.K, self.n, self.d, self.dev
        f64 = dict(dtype=torch.float64, device=dev)
        t0 = time.perf_counter()
        self.extra_calls = 0
        self._calls_dev.zero_()
        # captured slice moves hold the device pointers of the likelihood they were captured with
        # (for the GW likelihood: the event's tables), so every run captures them again
        self._graphs = None
        self.slice_graphs = self.slice_graphs_requested
        if live_u is None:
            live_u = torch.rand(K, d, generator=self.gen, **f64)
        live_u = live_u.to(**f64).contiguous()
        live_l, _ = self._loglike(live_u)
        o = torch.argsort(live_l, stable=True)
        live_u, live_l = live_u[o], live_l[o]

        cap = K * 64 + n * self.check_every
        dead_u = torch.empty(cap + 1, d, **f64)      # the last row takes the writes of non-dead slots
        dead_l = torch.empty(cap + 1, **f64)
        dead_ldx = torch.empty(cap + 1, **f64)
        dead_lx = torch.empty(cap + 1, **f64)
        n_acc = torch.zeros(max(1, min(max_iter, 1 << 16)), dtype=torch.int64, device=dev)
        n_dead = torch.zeros((), dtype=torch.int64, device=dev)
        ln_x = torch.zeros((), **f64)
        ln_z = torch.full((), -math.inf, **f64)
        stop = torch.zeros((), dtype=torch.bool, device=dev)
        pos = torch.arange(n, device=dev)
        ones_k = torch.ones(K, dtype=torch.bool, device=dev)
        it = 0
        synced_dead = 0
        while it < max_iter:
            if it % self.check_every == 0 and it > 0:
                if bool(stop):
                    break
                synced_dead = int(n_dead)
                if self.proposal == "gmc":   # step-length adaptation at the host's sync points
                    rate = float(self._gmc_rate)
                    self.gmc_scale *= 1.25 if rate > 0.5 else 0.8
            if synced_dead + n * (self.check_every + 1) > cap:      # grow the dead buffers
                synced_dead = int(n_dead)
                new_cap = max(2 * cap, synced_dead + n * (self.check_every + 1))
                dead_u, dead_l, dead_ldx, dead_lx = (torch.cat([b[:cap], torch.empty((new_cap - cap + 1,) + b.shape[1:], **f64)])
                                                     for b in (dead_u, dead_l, dead_ldx, dead_lx))
                cap = new_cap
            if it >= n_acc.numel():
                n_acc = torch.cat([n_acc, torch.zeros_like(n_acc)])
            lmin = live_l[0]
            cu = self._propose(it, live_u, live_l).to(**f64)
            cl, inside = self._loglike(cu)
            # iterations launched after the stop test passed (before the host reads the flag)
            # accept nothing and change nothing
            acc = inside & (cl >= lmin) & ~stop
            nacc = acc.sum()
            n_acc[it] = torch.where(stop, -1, nacc)
            # merged stable sort: by L (live before candidates on ties), then rejected first
            all_l = torch.cat([live_l, cl])
            all_u = torch.cat([live_u, cu])
            flag = torch.cat([ones_k, acc]).to(torch.int8)
            i1 = torch.argsort(all_l, stable=True)
            idx = i1[torch.argsort(flag[i1], stable=True)]
            sl, su = all_l[idx], all_u[idx]
            live_l, live_u = sl[n:].contiguous(), su[n:].contiguous()
            # dead points: merged positions [n - n', n), rank j = 1..n'
            j = pos - (n - nacc) + 1
            valid = j >= 1
            if self.volume == "order":
                dec = torch.where(j == 1, 1.0 / K, 1.0 / (K + nacc - j + 1).clamp(min=1).to(torch.float64))
            else:
                dec = torch.full((n,), 1.0 / K, **f64)
            dec = torch.where(valid, dec, torch.zeros_like(dec))
            cum = torch.cumsum(dec, 0)
            ldx = ln_x - (cum - dec) + torch.log(-torch.expm1(-dec))
            contrib = torch.where(valid, sl[:n] + ldx, torch.full_like(ldx, -math.inf))
            ln_z = torch.logaddexp(ln_z, torch.logsumexp(contrib, 0))
            dst = torch.where(valid, n_dead + j - 1, torch.full_like(j, cap))
            dead_l.index_copy_(0, dst, sl[:n])
            dead_u.index_copy_(0, dst, su[:n])
            dead_ldx.index_copy_(0, dst, ldx)
            dead_lx.index_copy_(0, dst, ln_x - cum)
            ln_x = ln_x - cum[-1]
            n_dead = n_dead + nacc
            bound = torch.logaddexp(ln_z, live_l[-1] + ln_x) - ln_z
            stop = stop | ((nacc > 0) & (bound <= eps))
            it += 1
        if dev.type == "cuda":
            torch.cuda.synchronize(dev)
        self.extra_calls += int(self._calls_dev) + (int(self._graphs.calls) if self._graphs is not None else 0)
        nd = int(n_dead)
        n_acc = n_acc[:it].cpu().numpy()
        n_acc = n_acc[n_acc >= 0]
        it = len(n_acc)
        # final live points: ascending, equal shares of the last volume
        lx = float(ln_x)
        share = lx - math.log(K)
        lz = float(ln_z)
        fin_l = live_l.cpu().numpy()
        lz = float(np.logaddexp(lz, np.logaddexp.reduce(fin_l + share))) if K else lz
        u = torch.cat([dead_u[:nd], live_u]).cpu().numpy()
        logl = np.concatenate([dead_l[:nd].cpu().numpy(), fin_l])
        log_dx = np.concatenate([dead_ldx[:nd].cpu().numpy(), np.full(K, share)])
        rem = np.array([lx + math.log((K - m) / K) if m < K else -math.inf for m in range(1, K + 1)])
        log_x = np.concatenate([dead_lx[:nd].cpu().numpy(), rem])
        log_w = logl + log_dx - lz
        w = np.exp(log_w)
        finite = np.isfinite(logl)
        h = float(np.sum(w[finite] * (logl[finite] - lz)))
        theta = self.transform(torch.tensor(u, **f64)).cpu().numpy() if len(u) else u
        return NSResult(u=u, theta=theta, logl=logl, log_dx=log_dx, log_x=log_x, logz=lz,
                        logz_err=math.sqrt(max(h, 0.0) / K), log_w=log_w, information=h, niter=it,
                        ncall=K + n * it + self.extra_calls, n_accepted=n_acc,
                        seconds=time.perf_counter() - t0, nlive=K)


def importance_logz(u_post, loglike, transform, dev, ncomp=16, ndraw=8_000_000, seed=7, scales=(1.0, 1.5, 2.5, 4.0)):
    """An evidence estimate independent of nested sampling, to check a run against: importance
    sampling in the unit cube with a Gaussian-mixture proposal fitted to posterior samples
    u_post[N, d] (ncomp components), mixed in equal parts with copies of it whose covariances
    are scaled by scales^2, ndraw draws. Coordinates whose posterior spread is that of a uniform
    draw (standard deviation above 0.27; a uniform one has 0.289, e.g. a parameter the likelihood
    ignores) are drawn uniformly instead, the mixture covering the others. Returns (ln Z,
    relative standard error of Z, effective sample size). A mode the posterior samples miss is
    missed here too."""
    from sklearn.mixture import GaussianMixture
    d_all = u_post.shape[1]
    flat = u_post.std(0) > 0.27
    keep = np.flatnonzero(~flat)
    gm = GaussianMixture(ncomp, covariance_type="full", reg_covar=1e-9, random_state=0,
                         max_iter=200).fit(u_post[:, keep])
    d = len(keep)
    keep_t = torch.tensor(keep, device=dev)
    flat_t = torch.tensor(np.flatnonzero(flat), device=dev)
    wts = torch.tensor(gm.weights_, device=dev)
    mus = torch.tensor(gm.means_, device=dev)
    chol = torch.linalg.cholesky(torch.tensor(gm.covariances_, device=dev))
    linv = torch.linalg.inv(chol)
    logdet = torch.log(torch.diagonal(chol, dim1=1, dim2=2)).sum(1)
    scales = torch.tensor(list(scales), dtype=torch.float64, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)

    def logq(v):
        """log density of the mixture part at v[B, d] (the uniform coordinates add 0)"""
        out = []
        for s in scales.tolist():
            y = torch.matmul(v[None] - mus[:, None], (linv / s).transpose(1, 2).contiguous())
            lp = -0.5 * (y * y).sum(-1) - (logdet + d * math.log(s))[:, None] - 0.5 * d * math.log(2 * math.pi)
            out.append(torch.logsumexp(lp + torch.log(wts)[:, None], 0))
        return torch.logsumexp(torch.stack(out), 0) - math.log(len(scales))

    lw, B = [], 131072
    for _ in range((ndraw + B - 1) // B):
        sc = scales[torch.randint(0, len(scales), (B,), generator=g, device=dev)]
        ci = torch.multinomial(wts, B, replacement=True, generator=g)
        z = torch.randn(B, d, generator=g, device=dev, dtype=torch.float64)
        v = mus[ci] + sc[:, None] * torch.matmul(chol[ci], z[..., None])[..., 0]
        u = torch.empty(B, d_all, dtype=torch.float64, device=dev)
        u[:, keep_t] = v
        if len(flat_t):
            u[:, flat_t] = torch.rand(B, len(flat_t), generator=g, device=dev, dtype=torch.float64)
        inside = ((u >= 0) & (u <= 1)).all(1)
        l = loglike(transform(u.clamp(0.0, 1.0)))
        l = torch.where(torch.isnan(l) | ~inside, torch.full_like(l, -math.inf), l)
        lw.append((l - logq(v)).cpu().numpy())
    lw = np.concatenate(lw)
    w = np.exp(lw - lw.max())
    return (lw.max() + math.log(w.mean()), w.std() / w.mean() / math.sqrt(len(w)),
            w.sum() ** 2 / (w * w).sum())
