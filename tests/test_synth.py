"""Pins of the seeded input generator (scanner simulator) against closed forms."""
import math

import mpmath as mp
import numpy as np
import pytest

from paper_1905_00934_amd import synth as S


def kn_by_quadrature(e_kev: float) -> float:
    """Integrate the Klein-Nishina differential cross-section over the sphere.

    d(sigma)/d(Omega) = r_e^2/2 P^2 (P + 1/P - sin^2 t), P = 1/(1 + a (1 - cos t));
    sigma / (2 pi r_e^2) = int_0^pi 1/2 P^2 (P + 1/P - sin^2 t) sin t dt.
    """
    mp.mp.dps = 30
    a = mp.mpf(e_kev) / mp.mpf(S.ELECTRON_REST_KEV)

    def integrand(t):
        P = 1 / (1 + a * (1 - mp.cos(t)))
        return 0.5 * P**2 * (P + 1 / P - mp.sin(t) ** 2) * mp.sin(t)

    return float(mp.quad(integrand, [0, mp.pi]))


@pytest.mark.parametrize("e", [20.0, 45.0, 60.0, 97.0, 130.0])
def test_klein_nishina_matches_angular_integral(e):
    assert S.klein_nishina(e) == pytest.approx(kn_by_quadrature(e), rel=1e-12)


@pytest.mark.parametrize("e", [1.0, 2.0, 5.0])
def test_klein_nishina_thomson_limit_series(e):
    a = e / S.ELECTRON_REST_KEV
    series = 4.0 / 3.0 * (1 - 2 * a + 26.0 / 5.0 * a**2 - 133.0 / 10.0 * a**3)
    assert S.klein_nishina(e) == pytest.approx(series, rel=1e-6)


def test_photoelectric_cubic_decay():
    e = S.energy_grid()
    fp = S.photoelectric(e)
    assert fp[e == 60.0][0] == 1.0
    np.testing.assert_allclose(fp * e**3, 60.0**3, rtol=1e-15)


def test_spectra_support_and_shape():
    sp = S.default_spectra()
    e = sp.energy_kev
    assert sp.n_bins == 111 and e[0] == 20.0 and e[-1] == 130.0
    assert np.all(sp.s_low[e >= 95] == 0) and np.all(sp.s_low[e < 95] > 0)
    assert np.all(sp.s_high[e >= 130] == 0) and np.all(sp.s_high[e < 130] > 0)
    mean_h = (sp.s_high * e).sum() / sp.s_high.sum()
    mean_l = (sp.s_low * e).sum() / sp.s_low.sum()
    assert 40 < mean_l < mean_h < 65


def test_ellipse_chord_is_circle_chord():
    sh = S.Shape("ellipse", 1.0, -2.0, 3.0, 3.0, 0.7, 1.0, 0.0)
    t = np.linspace(-2.9, 2.9, 11)
    th = 0.3
    o = np.stack([1.0 + t * math.cos(th), -2.0 + t * math.sin(th)], -1)
    d = np.tile([-math.sin(th), math.cos(th)], (t.size, 1))
    np.testing.assert_allclose(sh.chord(o, d), 2 * np.sqrt(9 - t**2), rtol=1e-13)


def test_ellipse_chord_along_axes():
    sh = S.Shape("ellipse", 0.5, 0.25, 4.0, 1.5, math.pi / 6, 1.0, 0.0)
    c, s = math.cos(sh.rot), math.sin(sh.rot)
    o = np.array([[0.5, 0.25], [0.5, 0.25]])
    d = np.array([[c, s], [-s, c]])
    np.testing.assert_allclose(sh.chord(o, d), [8.0, 3.0], rtol=1e-14)


def test_rectangle_chord_closed_form():
    hx, hy, rot = 2.0, 0.5, 0.4
    sh = S.Shape("rect", -1.0, 2.0, hx, hy, rot, 1.0, 0.0)
    for phi in (0.0, 0.1, 0.2, 1.0, 1.5):
        ang = rot + phi
        o = np.array([[-1.0, 2.0]])
        d = np.array([[math.cos(ang), math.sin(ang)]])
        with np.errstate(divide="ignore"):
            want = min(2 * hx / abs(math.cos(phi)) if math.cos(phi) else np.inf,
                       2 * hy / abs(math.sin(phi)) if math.sin(phi) else np.inf)
        assert sh.chord(o, d)[0] == pytest.approx(want, rel=1e-13)
    # A line that misses the rectangle.
    assert sh.chord(np.array([[10.0, 10.0]]), np.array([[1.0, 0.0]]))[0] == 0.0


def test_phantom_image_area_fractions():
    ph = S.Phantom([S.Shape("rect", 0.0, 0.0, 1.0, 1.0, 0.0, 0.5, 0.1)])
    xc, xp = ph.image(8, 8, 0.5, supersample=8)
    # The square covers exactly the central 4x4 pixels.
    assert xc.sum() * 0.25 == pytest.approx(0.5 * 4.0, rel=1e-12)
    assert np.count_nonzero(xc) == 16


def test_poisson_counts_statistics_and_seeding():
    lam = np.full(200_000, 50.0)
    a, b = S.poisson_counts(lam, 2 * lam, seed=5)
    assert abs(a.mean() - 50.0) < 5 * math.sqrt(50.0 / lam.size)
    assert abs(a.var() / 50.0 - 1.0) < 0.02
    assert abs(b.mean() - 100.0) < 5 * math.sqrt(100.0 / lam.size)
    a2, b2 = S.poisson_counts(lam, 2 * lam, seed=5)
    assert np.array_equal(a, a2) and np.array_equal(b, b2)
    a3, _ = S.poisson_counts(lam, 2 * lam, seed=6)
    assert not np.array_equal(a, a3)


def test_expected_counts_unattenuated_and_monochromatic():
    sp = S.default_spectra()
    z = np.zeros(3)
    lh, ll = S.expected_counts(sp, z, z, 1e5)
    np.testing.assert_allclose(lh, 1e5, rtol=1e-14)
    np.testing.assert_allclose(ll, 1e5, rtol=1e-14)
    mono = S.monochromatic_spectra(80.0, 40.0)
    ac, ap = np.array([0.5, 2.0]), np.array([0.1, 0.3])
    lh, ll = S.expected_counts(mono, ac, ap, 1.0)
    np.testing.assert_allclose(-np.log(lh), S.klein_nishina(80.0) * ac + S.photoelectric(80.0) * ap,
                               rtol=1e-14)


def test_luggage_phantom_structure():
    ph = S.luggage_phantom(0, 30, 2)
    steel = [s for s in ph.shapes if s.xc > 1.5]
    assert len(steel) == 2
    assert 25 <= len(ph.shapes) - 2 <= 30  # shell is two shapes
    for s in ph.shapes:
        x0, x1, y0, y1 = s.bbox()
        assert max(abs(x0), abs(x1), abs(y0), abs(y1)) < 25.6
