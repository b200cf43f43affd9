"""Pins of the oracle's CDM-FBP baseline and initial image (Sec. 2 CDM, Sec. 4 set-up):
constrained per-ray decomposition (a >= 0) and filtered backprojection."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle as O
from paper_1905_00934_amd import synth as S


@pytest.mark.parametrize("delta", [0.25, 0.0953])
def test_ramlak_kernel_is_sampled_band_limited_ramp(delta):
    """h(n delta) = integral of |w| exp(2 pi i w n delta) over |w| <= 1/(2 delta)."""
    P = 64
    h = O.ramlak_kernel(P, delta)
    W = 1.0 / (2.0 * delta)
    for n in range(-7, 8):
        want = 2.0 * quad(lambda w: w * math.cos(2 * math.pi * w * n * delta), 0.0, W,
                          limit=200, epsabs=1e-13, epsrel=1e-12)[0]
        assert h[n % P] == pytest.approx(want, rel=1e-9, abs=1e-9 / delta ** 2)


def _disk_case(kind, cx=1.5, cy=-2.0, r=8.0, mu=0.3):
    if kind == "parallel":
        g = S.geometry("parallel", 128, 128, 0.25, 180, 183, 0.25)
    else:
        g = S.geometry("fan", 128, 128, 0.25, 360, 256, 0.3, src_iso_cm=60.0, src_det_cm=100.0)
    ph = S.Phantom([S.Shape("ellipse", cx, cy, r, r, 0.0, mu, 0.0)])
    ac, _ = ph.line_integrals(g)
    orc = O.Oracle(g, S.default_spectra())
    img = orc.fbp(ac)
    xs = (np.arange(128) - 63.5) * 0.25
    X, Y = np.meshgrid(xs, xs)
    dist = np.hypot(X - cx, Y - cy)
    return img, dist, X, Y


@pytest.mark.parametrize("kind", ["parallel", "fan"])
def test_fbp_reconstructs_uniform_disk(kind):
    img, dist, X, Y = _disk_case(kind)
    inside = dist < 8.0 - 1.0
    outside = dist > 8.0 + 1.0
    assert abs(img[inside].mean() / 0.3 - 1.0) < 0.01
    assert np.abs(img[inside] - 0.3).max() < 0.03
    assert np.abs(img[outside]).mean() < 0.003
    # The disk is where it should be (a flipped axis or angle would move it).
    m = img > 0.15
    assert abs(X[m].mean() - 1.5) < 0.25 and abs(Y[m].mean() + 2.0) < 0.25


def test_fan_fbp_off_centre_disk_near_the_source():
    """A disk 10 cm off the centre with the source 40 cm away: the distance weighting
    U^-2 varies by +-30 % over the turn, so a wrong power of U biases the disk."""
    g = S.geometry("fan", 128, 128, 0.25, 360, 400, 0.25, src_iso_cm=40.0, src_det_cm=80.0)
    cx, cy, r, mu = 9.0, 5.0, 3.0, 0.5
    ph = S.Phantom([S.Shape("ellipse", cx, cy, r, r, 0.0, mu, 0.0)])
    ac, _ = ph.line_integrals(g)
    img = O.Oracle(g, S.default_spectra()).fbp(ac)
    xs = (np.arange(128) - 63.5) * 0.25
    X, Y = np.meshgrid(xs, xs)
    d = np.hypot(X - cx, Y - cy)
    assert abs(img[d < r - 0.75].mean() / mu - 1.0) < 0.01
    assert np.abs(img[d < r - 0.75] - mu).max() < 0.05 * mu


def test_fbp_is_linear_and_scale_free():
    img1, *_ = _disk_case("fan", mu=0.3)
    img2, *_ = _disk_case("fan", mu=0.6)
    np.testing.assert_allclose(img2, 2.0 * img1, rtol=1e-12, atol=1e-12)


def _rays(n=200, seed=0, lo=(0.0, 0.0), hi=(8.0, 3.0)):
    """Line integrals in the range where the expected counts stay above one photon."""
    rng = np.random.default_rng(seed)
    ac = rng.uniform(lo[0], hi[0], n)
    ap = rng.uniform(lo[1], hi[1], n)
    return ac, ap


def test_cdm_recovers_nonnegative_noiseless_rays():
    spec = S.default_spectra()
    orc = O.Oracle(S.geometry("parallel", 4, 4, 1.0, 1, 4, 1.0), spec)
    ac, ap = _rays()
    ac[:10] = 0.0   # on the boundary
    ap[10:20] = 0.0
    lh, ll = S.expected_counts(spec, ac, ap, 1e5)
    mh, wh = O.ingest(lh, 1e5)
    ml, wl = O.ingest(ll, 1e5)
    c, p = orc.cdm(mh, ml, wh, wl, iters=80)
    assert np.all(c >= 0) and np.all(p >= 0)
    np.testing.assert_allclose(c, ac, atol=1e-6)
    np.testing.assert_allclose(p, ap, atol=1e-5)


def test_cdm_kkt_and_agreement_with_udm():
    """Noisy rays: at the CDM solution the gradient of the data cost vanishes along
    free coordinates and points into the feasible set along active ones; where no
    constraint is active CDM equals the unconstrained decomposition (rho = 0)."""
    spec = S.default_spectra()
    orc = O.Oracle(S.geometry("parallel", 4, 4, 1.0, 1, 4, 1.0), spec)
    ac, ap = _rays(seed=3, lo=(0.0, 0.0), hi=(3.0, 0.5))  # thin rays: noise drives a_p < 0
    lh, ll = S.expected_counts(spec, ac, ap, 2e4)
    ch, cl = S.poisson_counts(lh, ll, 9)
    mh, wh = O.ingest(ch, 2e4)
    ml, wl = O.ingest(cl, 2e4)
    c, p = orc.cdm(mh, ml, wh, wl, iters=200)
    fh, fl, gh, gl = orc.forward(c, p)
    rh, rl = wh * (fh - mh), wl * (fl - ml)
    Gc = rh * gh[..., 0] + rl * gl[..., 0]
    Gp = rh * gh[..., 1] + rl * gl[..., 1]
    # Size of the gradient's terms (an exactly fitted ray has a gradient at rounding level).
    tol = 1e-6 * (np.abs(rh) * np.abs(gh).sum(-1) + np.abs(rl) * np.abs(gl).sum(-1)) + 1e-12
    act_p = p == 0.0
    assert act_p.sum() > 5   # the constraint is active on some rays
    assert np.all(Gp[act_p] >= -tol[act_p])
    assert np.all(np.abs(Gp[~act_p]) <= tol[~act_p])
    free_c = c > 0.0
    assert np.all(np.abs(Gc[free_c]) <= tol[free_c])
    # Interior rays: the unconstrained decomposition lands on the same point.
    c0, p0 = orc.linearised(mh, ml)
    cu, pu, _ = orc.udm(mh, ml, wh, wl, None, None, 0.0, 0.0, 200, c0, p0)
    inner = (cu > 1e-3) & (pu > 1e-3)
    assert inner.sum() > 20
    np.testing.assert_allclose(c[inner], cu[inner], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(p[inner], pu[inner], rtol=1e-6, atol=1e-9)


def test_cdm_fbp_start_and_admm_init_from_image():
    pr = S.tiny_problem(0)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    (ac, ap), x = orc.cdm_fbp(mh, ml, wh, wl, 20)
    x0 = orc.cdm_fbp_start(mh, ml, wh, wl, 20)
    np.testing.assert_allclose(x0[0], x[0], rtol=0, atol=0)
    np.testing.assert_allclose(x0[1], x[0] * ap.sum() / ac.sum(), rtol=1e-14)
    # The CDM-FBP Compton image is close to the truth (a baseline, not a pin of quality).
    assert O.xi_db(x[0], pr.x_true[0]) < -10
    st = orc.admm_init(mh, ml, wh, wl, O.Params(), x0=x0)
    for b in range(2):
        np.testing.assert_allclose(st.Rx[b], orc.project(x0[b], count=None), rtol=1e-14)
        np.testing.assert_allclose(st.y[b], O.D(x0[b]), rtol=1e-14)
    np.testing.assert_array_equal(st.z, x0)
    assert not np.any(st.ua) and not np.any(st.uy) and not np.any(st.uz)
