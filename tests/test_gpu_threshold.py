"""GPU parity of the density thresholding of Sec. 5 against the oracle, through
the C ABI: the strategy based on the density values (Sec. 5.1), the rounding
near 0 and 1, the angle condition (Sec. 5.2) and the smooth Heaviside
projection with its volume-preserving threshold (Sec. 5.4).

The top-k selection and the rounding are exact (0/1 choices from FP64
comparisons): compared bit for bit.  The cosine of the angle is a quotient of
three sums of n products; each sum in another order than the oracle's is
within n eps of the sum of the magnitudes, which by Cauchy-Schwarz bounds the
cosine's difference by 4 n eps.  The Heaviside threshold eta is a root found to
|f| <= 1e-13 sum(rho) or |delta eta| <= 1e-14 on both sides, with sums in
different orders: the two agree to 1e-10 (the oracle's own pin against
scipy's brentq), and h is compared with the oracle's h at the library's eta
to a few ulps of tanh (1e-14)."""

import math

import numpy as np
import pytest

from oracle import threshold as T
from tests.helpers import need_gpu

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _densities(n, seed, decimals=None):
    rng = np.random.default_rng(seed)
    rho = np.clip(rng.beta(0.7, 1.2, n), 0.0, 1.0)
    if decimals is not None:
        rho = np.round(rho, decimals)  # many equal values
    return rho


@pytest.mark.parametrize("n,seed,vfrac,dec", [
    (1, 0, 1.0, None), (1, 1, 0.0, None), (7, 2, 0.5, 1), (255, 3, 0.3, None),
    (256, 4, 0.25, 2), (257, 5, 0.3, 1), (5000, 6, 0.12, 2), (70001, 7, 0.4, None),
    (70001, 8, 0.4, 1)])
def test_density_threshold_matches_oracle(n, seed, vfrac, dec):
    need_gpu()
    from paper_2311_05595_amd import api
    lp = api.LP(n)
    rho = _densities(n, seed, dec)
    out = lp.density_threshold(rho, vfrac)
    assert np.array_equal(out, T.density_threshold(rho, vfrac))
    lp.close()


def test_select_top_extremes_and_errors():
    need_gpu()
    from paper_2311_05595_amd import api
    from paper_2311_05595_amd._abi import MGCGError
    n = 1000
    lp = api.LP(n)
    v = np.round(np.random.default_rng(9).standard_normal(n), 1)
    v[::5] = 0.0
    v[1::5] = -0.0   # one key for both zeros: ties in index order
    for k in (0, 1, 499, 500, 999, 1000):
        ref = np.zeros(n)
        ref[sorted(range(n), key=lambda i: (-v[i], i))[:k]] = 1.0
        assert np.array_equal(lp.select_top(v, k), ref), k
    with pytest.raises(MGCGError):
        lp.select_top(v, n + 1)
    bad = v.copy()
    bad[3] = np.nan
    with pytest.raises(MGCGError):
        lp.select_top(bad, 10)
    # still usable
    assert lp.select_top(v, 10).sum() == 10
    lp.close()


def test_pre_round_matches_oracle():
    need_gpu()
    import torch
    from paper_2311_05595_amd import api
    n = 3001
    rho = _densities(n, 10, 3)
    rho[:6] = [0.05, 0.0500001, 0.95, 0.9499999, 0.0, 1.0]
    lp = api.LP(n)
    assert np.array_equal(lp.pre_round(rho), T.pre_round(rho))
    d = torch.tensor(rho, device="cuda")
    lp.pre_round(d, out=d)   # in place on the device
    assert np.array_equal(d.cpu().numpy(), T.pre_round(rho))
    lp.close()


@pytest.mark.parametrize("n,seed", [(1, 0), (300, 1), (70001, 2)])
def test_angle_cos_matches_oracle(n, seed):
    need_gpu()
    from paper_2311_05595_amd import api
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(n)
    d = -g + 0.7 * rng.standard_normal(n)
    lp = api.LP(n)
    c = lp.angle_cos(g, d)
    assert abs(c - T.angle_cos(g, d)) <= 4 * n * EPS + 1e-300
    assert (c > math.cos(math.radians(89.9))) == T.angle_ok(g, d)
    lp.close()


@pytest.mark.parametrize("n,seed,beta", [(1000, 0, 1.0), (5000, 1, 2.0), (70001, 2, 16.0),
                                         (70001, 3, 100.0), (257, 4, 8.0)])
def test_heaviside_matches_oracle(n, seed, beta):
    need_gpu()
    from paper_2311_05595_amd import api
    rho = _densities(n, seed)
    lp = api.LP(n)
    h, eta, it = lp.heaviside(rho, beta)
    eta_o = T.eta_newton(rho, beta)
    assert abs(eta - eta_o) <= 1e-10
    assert 1 <= it <= 100
    assert np.abs(h - T.heaviside(rho, beta, eta)).max() <= 1e-14
    assert abs(h.sum() - rho.sum()) <= 1e-9 * rho.sum()
    with pytest.raises(Exception):
        lp.heaviside(rho, 0.0)
    lp.close()


def test_threshold_full_size_device_memory():
    """The density lattice of the 64x32x32 mesh with 4^3 sub-elements per
    element (4,194,304 densities) in device memory: the top-k rule checked by
    its properties (exactly k ones, no zero above a one, the tied values at the
    threshold taken in index order), the host path's bits, and the Heaviside
    projection against the oracle's threshold and sampled values."""
    need_gpu()
    import torch
    from paper_2311_05595_amd import api
    n = 64 * 32 * 32 * 64
    rho = _densities(n, 11, 3)
    lp = api.LP(n)
    d = torch.tensor(rho, device="cuda")
    vfrac = 0.3
    k = int(math.floor(vfrac * n))
    out = lp.density_threshold(d, vfrac).cpu().numpy()
    assert out.sum() == k and np.all((out == 0.0) | (out == 1.0))
    t = rho[out == 1.0].min()
    assert rho[out == 0.0].max() <= t
    tied = np.flatnonzero(rho == t)
    sel = out[tied]
    m = int(sel.sum())
    assert np.all(sel[:m] == 1.0) and np.all(sel[m:] == 0.0)
    assert np.array_equal(lp.density_threshold(rho, vfrac), out)
    beta = 8.0
    h, eta, it = lp.heaviside(d, beta)
    assert abs(eta - T.eta_newton(rho, beta)) <= 1e-10
    h = h.cpu().numpy()
    idx = np.random.default_rng(12).choice(n, 4096, replace=False)
    assert np.abs(h[idx] - T.heaviside(rho[idx], beta, eta)).max() <= 1e-14
    assert abs(h.sum() - rho.sum()) <= 1e-9 * rho.sum()
    c = lp.angle_cos(d - 0.5, torch.tensor(0.5 - rho, device="cuda"))
    assert abs(c - T.angle_cos(rho - 0.5, 0.5 - rho)) <= 4 * n * EPS
    lp.close()


def _lagrangian_case(n, seed, kind):
    rng = np.random.default_rng(seed)
    if kind == "bind":
        rho = np.full(n, 0.5)
        g = np.where(np.arange(n) % 2 == 0, 1e-6, -1e-6)
        rho[0], g[0] = 0.94, -1e3
        return rho, g
    if kind == "box":   # no safeguard can bind: the angle condition decides
        rho = rng.uniform(0.3, 0.7, n)
        g = rng.standard_normal(n) * np.exp(3.0 * rng.standard_normal(n))
        return rho, g
    rho = T.pre_round(rng.beta(0.6, 0.6, n))
    g = rng.standard_normal(n) * rng.exponential(1.0, n) ** 3
    g[rng.random(n) < 0.05] = 0.0
    if kind == "ties":
        rho, g = np.round(rho, 1), np.round(g, 1)
    return rho, g


@pytest.mark.parametrize("n,seed,kind", [
    (1, 0, "mixed"), (2, 1, "box"), (7, 2, "mixed"), (300, 3, "mixed"), (257, 4, "ties"),
    (2000, 5, "box"), (3001, 0, "bind"), (6001, 0, "bind"), (1500, 6, "mixed")])
def test_lagrangian_threshold_matches_oracle(n, seed, kind):
    """alpha~ is one of the alpha_i, the same quotient on both sides: compared
    exactly, and rho~ (bounds, or rho - alpha~ g rounded after the product)
    bit for bit."""
    need_gpu()
    from paper_2311_05595_amd import api
    rho, g = _lagrangian_case(n, seed, kind)
    lp = api.LP(n)
    out, a = lp.lagrangian_threshold(rho, g)
    ref, a_o = T.lagrangian_threshold(rho, g)
    assert a == a_o
    assert np.array_equal(out, ref)
    lp.close()


def test_lagrangian_threshold_degenerate():
    """No gradient, or every density already at the bound it would reach:
    alpha~ = 0 and rho~ = rho."""
    need_gpu()
    from paper_2311_05595_amd import api
    n = 513
    lp = api.LP(n)
    rho = np.random.default_rng(3).uniform(0, 1, n)
    out, a = lp.lagrangian_threshold(rho, np.zeros(n))
    assert a == 0.0 and np.array_equal(out, rho)
    rho = np.where(np.arange(n) % 2 == 0, 0.0, 1.0)
    g = np.where(rho == 0.0, 1.0, -1.0)
    out, a = lp.lagrangian_threshold(rho, g)
    assert a == 0.0 and np.array_equal(out, rho)
    lp.close()


def test_lagrangian_threshold_full_size():
    """4,194,304 densities in device memory, heavy-tailed gradients: alpha~
    passes the angle test and the safeguards, and the next larger alpha_i
    breaks one of them (the cosine from its closed form,
    sum g^2 m / (|g| sqrt(sum g^2 m^2)), m_i = min(alpha, alpha_i))."""
    need_gpu()
    import torch
    from paper_2311_05595_amd import api
    n = 64 * 32 * 32 * 64
    rng = np.random.default_rng(13)
    rho = T.pre_round(np.clip(rng.beta(0.7, 1.2, n), 0.0, 1.0))
    g = rng.standard_normal(n) * np.exp(2.0 * rng.standard_normal(n))
    lp = api.LP(n)
    out, a = lp.lagrangian_threshold(torch.tensor(rho, device="cuda"),
                                     torch.tensor(g, device="cuda"))
    out = out.cpu().numpy()
    alpha = T.lagrangian_alphas(rho, g)
    w = g * g
    cmax = math.cos(math.radians(89.9))
    bad = ((g < 0) & (rho < 0.3)) | ((g > 0) & (rho > 0.7))
    viol = alpha[bad].min() if bad.any() else np.inf

    def cos(x):
        m = np.minimum(x, alpha)
        return np.sum(w * m) / (math.sqrt(w.sum()) * math.sqrt(np.sum(w * m * m)))

    assert a > 0.0 and a < viol and cos(a) > cmax
    nxt = alpha[np.isfinite(alpha) & (alpha > a)].min()
    assert nxt >= viol or cos(nxt) <= cmax
    idx = np.random.default_rng(14).choice(n, 4096, replace=False)
    assert np.array_equal(out[idx], T.lagrangian_step(rho[idx], g[idx], a))
    lp.close()


def test_lagrangian_threshold_all_equal_steps():
    """Every density at the same step (rho = 0.5, g = 1): the bracket keeps
    all of them inside, more than the compaction's scratch holds, so the
    search stays on the full arrays; alpha~ = 0.5 and every density goes to 0."""
    need_gpu()
    from paper_2311_05595_amd import api
    n = 1000
    rho, g = np.full(n, 0.5), np.ones(n)
    lp = api.LP(n)
    out, a = lp.lagrangian_threshold(rho, g)
    ref, a_o = T.lagrangian_threshold(rho, g)
    assert a == a_o == 0.5 and np.array_equal(out, ref) and np.all(out == 0.0)
    lp.close()


@pytest.mark.parametrize("value", [0.0, 0.3, 1.0])
def test_heaviside_constant_densities(value):
    """Equal densities: for 0 every eta keeps the (zero) volume and Newton
    stops at its start; otherwise eta is where h(value) = value."""
    need_gpu()
    from paper_2311_05595_amd import api
    n = 777
    rho = np.full(n, value)
    lp = api.LP(n)
    h, eta, it = lp.heaviside(rho, 8.0)
    eta_o = T.eta_newton(rho, 8.0)
    assert abs(eta - eta_o) <= 1e-10
    assert np.abs(h - T.heaviside(rho, 8.0, eta)).max() <= 1e-14
    assert abs(h.sum() - rho.sum()) <= 1e-9 * max(rho.sum(), 1.0)
    lp.close()
