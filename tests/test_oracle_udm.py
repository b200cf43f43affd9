"""Pins of the oracle's forward transform f (Eq. (3)) and per-ray decomposition (Eq. (13))."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from paper_1905_00934_amd import synth as S

GEOM = S.geometry("parallel", 4, 4, 1.0, 2, 4, 1.0)


def _orc(spec=None):
    return O.Oracle(GEOM, S.default_spectra() if spec is None else spec)


def test_forward_monochromatic_is_linear():
    spec = S.monochromatic_spectra(80.0, 40.0)
    orc = _orc(spec)
    rng = np.random.default_rng(0)
    ac, ap = rng.uniform(0, 10, 50), rng.uniform(0, 3, 50)
    fh, fl, gh, gl = orc.forward(ac, ap)
    kh, ph = S.klein_nishina(80.0), S.photoelectric(80.0)
    kl, pl = S.klein_nishina(40.0), S.photoelectric(40.0)
    np.testing.assert_allclose(fh, kh * ac + ph * ap, rtol=1e-13)
    np.testing.assert_allclose(fl, kl * ac + pl * ap, rtol=1e-13)
    np.testing.assert_allclose(gh[:, 0], kh, rtol=1e-13)
    np.testing.assert_allclose(gl[:, 1], pl, rtol=1e-13)


def _f_mp(spec_s, spec, ac, ap):
    mp.mp.dps = 40
    tot = mp.mpf(0)
    acc = mp.mpf(0)
    for k in range(spec.n_bins):
        s = mp.mpf(float(spec_s[k]))
        tot += s
        acc += s * mp.exp(-mp.mpf(float(spec.f_kn[k])) * mp.mpf(ac)
                          - mp.mpf(float(spec.f_p[k])) * mp.mpf(ap))
    return float(-mp.log(acc / tot))


@pytest.mark.parametrize("ac,ap", [(0.0, 0.0), (1.5, 0.2), (9.0, 3.0), (12.0, 25.0),
                                   (40.0, 200.0), (-0.5, -0.05)])
def test_forward_matches_high_precision_sum(ac, ap):
    spec = S.default_spectra()
    orc = _orc(spec)
    fh, fl, _, _ = orc.forward(np.array([ac]), np.array([ap]))
    assert fh[0] == pytest.approx(_f_mp(spec.s_high, spec, ac, ap), rel=1e-13, abs=1e-14)
    assert fl[0] == pytest.approx(_f_mp(spec.s_low, spec, ac, ap), rel=1e-13, abs=1e-14)


def test_forward_gradient_finite_differences():
    orc = _orc()
    rng = np.random.default_rng(1)
    ac, ap = rng.uniform(0, 10, 20), rng.uniform(0, 5, 20)
    _, _, gh, gl = orc.forward(ac, ap)
    h = 1e-6
    for k, (dc, dp) in enumerate(((h, 0.0), (0.0, h))):
        fph, fpl, _, _ = orc.forward(ac + dc, ap + dp)
        fmh, fml, _, _ = orc.forward(ac - dc, ap - dp)
        np.testing.assert_allclose(gh[:, k], (fph - fmh) / (2 * h), rtol=1e-7)
        np.testing.assert_allclose(gl[:, k], (fpl - fml) / (2 * h), rtol=1e-7)


@pytest.mark.parametrize("rho", [(0.0, 0.0), (0.3, 2.0)])
def test_udm_monochromatic_is_ridge_least_squares(rho):
    """With single-line spectra f(a) = J a, so Eq. (13) is a weighted ridge problem."""
    spec = S.monochromatic_spectra(80.0, 40.0)
    orc = _orc(spec)
    J = np.array([[S.klein_nishina(80.0), S.photoelectric(80.0)],
                  [S.klein_nishina(40.0), S.photoelectric(40.0)]])
    rng = np.random.default_rng(2)
    n = 40
    mh, ml = rng.uniform(0, 8, n), rng.uniform(0, 12, n)
    wh, wl = rng.uniform(0.01, 1, n), rng.uniform(0.01, 1, n)
    vc, vp = rng.uniform(0, 5, n), rng.uniform(0, 2, n)
    ac, ap, _ = orc.udm(mh, ml, wh, wl, vc, vp, rho[0], rho[1], 30, np.zeros(n), np.zeros(n))
    for i in range(n):
        W = np.diag([wh[i], wl[i]])
        A = J.T @ W @ J + np.diag(rho)
        rhs = J.T @ W @ np.array([mh[i], ml[i]]) + np.array(rho) * np.array([vc[i], vp[i]])
        want = np.linalg.solve(A, rhs)
        # Accept decisions compare costs, so the step resolution is limited by rounding of
        # Phi near its minimum.
        np.testing.assert_allclose([ac[i], ap[i]], want, rtol=1e-10, atol=1e-10)


def test_udm_recovers_noiseless_polychromatic_line_integrals():
    """Forward-simulate exact data on a grid covering the phantoms' range, decompose
    with rho = 0 from the linearised start, and recover the line integrals."""
    spec = S.default_spectra()
    orc = _orc(spec)
    gc, gp = np.meshgrid(np.linspace(0, 12, 13), np.linspace(0, 25, 11))
    ac_true, ap_true = gc.ravel(), gp.ravel()
    i0 = 1e5
    lh, ll = S.expected_counts(spec, ac_true, ap_true, i0)
    mh, ml = -np.log(lh / i0), -np.log(ll / i0)
    wh, wl = lh / i0, ll / i0
    a0c, a0p = orc.linearised(mh, ml)
    ac, ap, _ = orc.udm(mh, ml, wh, wl, None, None, 0.0, 0.0, 30, a0c, a0p)
    np.testing.assert_allclose(ac, ac_true, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(ap, ap_true, rtol=1e-10, atol=1e-10)


def test_udm_reaches_brute_force_minimum_with_noise_and_rho():
    spec = S.default_spectra()
    orc = _orc(spec)
    rng = np.random.default_rng(3)
    n = 25
    ac_true, ap_true = rng.uniform(0.5, 8, n), rng.uniform(0.0, 4, n)
    i0 = 2e5
    lh, ll = S.expected_counts(spec, ac_true, ap_true, i0)
    ch, cl = S.poisson_counts(lh, ll, seed=9)
    mh, ml = np.log(i0 / np.maximum(ch, 1)), np.log(i0 / np.maximum(cl, 1))
    wh, wl = ch / i0, cl / i0
    vc = ac_true + rng.normal(0, 0.2, n)
    vp = ap_true + rng.normal(0, 0.2, n)
    rc, rp = 0.02, 0.05
    a0c, a0p = orc.linearised(mh, ml)
    ac, ap, phi = orc.udm(mh, ml, wh, wl, vc, vp, rc, rp, 60, a0c, a0p)

    def cost(a, i):
        # Eq. (13) for ray i, evaluated with a plain sum over energy bins.
        out = 0.5 * (rc * (a[0] - vc[i]) ** 2 + rp * (a[1] - vp[i]) ** 2)
        for s, m, w in ((spec.s_high, mh[i], wh[i]), (spec.s_low, ml[i], wl[i])):
            t = np.sum(s * np.exp(-spec.f_kn * a[0] - spec.f_p * a[1])) / s.sum()
            out += 0.5 * w * (-math.log(t) - m) ** 2
        return out

    for i in range(n):
        grid = [(c, p) for c in np.linspace(0, 10, 41) for p in np.linspace(-1, 6, 41)]
        start = min(grid, key=lambda a: cost(a, i))
        res = minimize(lambda a: cost(a, i), start, method="Nelder-Mead",
                       options=dict(xatol=1e-12, fatol=1e-15, maxiter=20000))
        assert phi[i] == pytest.approx(cost((ac[i], ap[i]), i), rel=1e-12)
        assert phi[i] <= res.fun * (1 + 1e-10) + 1e-15


def test_udm_counts_forward_evaluations():
    orc = _orc()
    for m in (1, 2, 5):
        before = orc.counts["f"]
        orc.udm(np.ones(3), np.ones(3), np.ones(3), np.ones(3), np.ones(3), np.ones(3), 0.1,
                0.1, m, np.zeros(3), np.zeros(3))
        assert orc.counts["f"] - before == 2 * (m + 1)


def test_udm_replayed_decisions():
    """Replaying accept decisions: the oracle's own decisions reproduce its unforced run
    bit for bit with no disagreement recorded; the opposite decisions are followed, and
    each one is reported far from a single-precision near-tie."""
    orc = _orc()
    rng = np.random.default_rng(11)
    n = 400
    ac_t, ap_t = rng.uniform(0, 12, n), rng.uniform(0, 10, n)
    fh, fl, _, _ = orc.forward(ac_t, ap_t)
    mh, ml = fh + rng.normal(0, 0.02, n), fl + rng.normal(0, 0.02, n)
    wh, wl = rng.uniform(0.05, 1, n), rng.uniform(0.05, 1, n)
    vc, vp = ac_t + rng.normal(0, 0.3, n), ap_t + rng.normal(0, 0.3, n)
    a0c, a0p = ac_t + rng.normal(0, 1.0, n), ap_t + rng.normal(0, 1.0, n)
    args = (mh, ml, wh, wl, vc, vp, 1e-3, 2e-3, 1)
    # One LM iteration: it accepted exactly where a moved.
    c1, p1, phi1 = orc.udm(*args, a0c, a0p)
    own = ((c1 != a0c) | (p1 != a0p)).astype(np.uint8)
    assert 0 < own.sum() < n
    ties = []
    c2, p2, phi2 = orc.udm(*args, a0c, a0p, force=own, ties=ties)
    np.testing.assert_array_equal(c2, c1)
    np.testing.assert_array_equal(p2, p1)
    assert not ties[0].any()
    # The opposite decisions: accepted steps are undone, rejected ones taken.
    ties = []
    c3, p3, _ = orc.udm(*args, a0c, a0p, force=1 - own, ties=ties)
    np.testing.assert_array_equal(c3[own == 1], a0c[own == 1])
    assert np.all((c3 != a0c)[own == 0])
    assert np.all(ties[0] > 0)
    # A real disagreement is thousands of rounding scales away from a tie.
    assert np.median(ties[0]) > 1e3
