"""Pins of the oracle's linear operators (R, R^T, D, D^T) and elementwise proxes.

Each expected value comes from a closed form, an explicit matrix, an analytic
line integral or a scalar minimisation, never from the oracle itself.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle as O
from paper_1905_00934_amd import synth as S


def _axis_geom():
    return S.geometry("parallel", 16, 16, 1.0, 2, 16, 1.0)  # views at 0 and pi/2


def test_axis_aligned_views_are_column_and_row_sums():
    g = _axis_geom()
    orc = O.Oracle(g, S.default_spectra())
    X = np.random.default_rng(1).uniform(0, 1, (16, 16))
    sino = orc.project(X)
    # theta = 0: vertical lines through the pixel centres x = x_b -> column sums.
    np.testing.assert_allclose(sino[0], X.sum(axis=0), rtol=1e-13)
    # theta = pi/2: horizontal lines y = y_b -> row sums.
    np.testing.assert_allclose(sino[1], X.sum(axis=1), rtol=1e-13)


def test_constant_image_full_chord():
    g = S.geometry("parallel", 20, 12, 0.5, 2, 12, 0.5)
    orc = O.Oracle(g, S.default_spectra())
    sino = orc.project(np.ones((12, 20)))
    # Vertical rays (theta = 0) cross the 12 rows: length 12 * 0.5 = 6 cm.
    np.testing.assert_allclose(sino[0], 6.0, rtol=1e-14)


def _linear_image(nx, ny, c):
    j, i = np.mgrid[0:ny, 0:nx]
    return c[0] + c[1] * i + c[2] * j


@pytest.mark.parametrize("kind", ["parallel", "fan"])
def test_linear_image_projection_is_exact_line_integral(kind):
    """Linear interpolation reproduces a linear image exactly, so the Joseph sum of a
    ray that stays inside the image equals the midpoint rule of the line integral of
    a linear function, i.e. (number of samples) x (step length) x (value at the
    image centre line)."""
    nx, ny, d = 24, 16, 0.7
    if kind == "parallel":
        g = S.geometry("parallel", nx, ny, d, 36, 41, 0.35)
    else:
        g = S.geometry("fan", nx, ny, d, 36, 61, 0.6, src_iso_cm=40.0, src_det_cm=70.0)
    orc = O.Oracle(g, S.default_spectra())
    c = (0.3, 0.011, -0.023)
    sino = orc.project(_linear_image(nx, ny, c))
    o, u = S.ray_lines(g)
    checked = 0
    for v in range(g["n_views"]):
        for b in range(g["n_det"]):
            (ox, oy), (dx, dy) = o[v, b], u[v, b]
            if abs(dx) >= abs(dy):
                s = dy / dx
                y0 = oy + (0.0 - ox) * s
                phis = [(oy + (x - ox) * s) / d + (ny - 1) / 2
                        for x in ((np.arange(nx) - (nx - 1) / 2) * d)]
                if min(phis) < 0 or max(phis) > ny - 1:
                    continue
                want = d * math.sqrt(1 + s * s) * nx * (
                    c[0] + c[1] * (nx - 1) / 2 + c[2] * (y0 / d + (ny - 1) / 2))
            else:
                s = dx / dy
                x0 = ox + (0.0 - oy) * s
                psis = [(ox + (y - oy) * s) / d + (nx - 1) / 2
                        for y in ((np.arange(ny) - (ny - 1) / 2) * d)]
                if min(psis) < 0 or max(psis) > nx - 1:
                    continue
                want = d * math.sqrt(1 + s * s) * ny * (
                    c[0] + c[1] * (x0 / d + (nx - 1) / 2) + c[2] * (ny - 1) / 2)
            assert sino[v, b] == pytest.approx(want, rel=1e-12, abs=1e-12)
            checked += 1
    assert checked > 200


@pytest.mark.parametrize("kind", ["parallel", "fan"])
def test_projection_of_disk_matches_analytic_chords(kind):
    """Joseph projection of an area-weighted off-centre disk against the exact chord
    lengths 2 sqrt(r^2 - t^2); the tolerance is a discretisation bound."""
    n, d = 64, 0.5
    if kind == "parallel":
        g = S.geometry("parallel", n, n, d, 90, 101, 0.45)
    else:
        g = S.fan_geometry_fov(n, 90, 128, fov_cm=n * d, src_iso_cm=40.0, src_det_cm=70.0)
    ph = S.Phantom([S.Shape("ellipse", 3.0, -4.5, 10.0, 10.0, 0.0, 1.0, 0.0)])
    img, _ = ph.image(n, n, d, supersample=16)
    orc = O.Oracle(g, S.default_spectra())
    sino = orc.project(img)
    exact, _ = ph.line_integrals(g)
    inner = exact > 2 * math.sqrt(10.0**2 - (10.0 - 2 * d) ** 2)
    err = np.linalg.norm(sino[inner] - exact[inner]) / np.linalg.norm(exact[inner])
    assert err < 0.005
    # Rays at least two pixels inside the rim see the edge blur of one pixel only.
    assert np.max(np.abs(sino - exact)[inner]) < d


def test_backprojection_is_transpose_of_explicit_matrix():
    g = S.geometry("fan", 12, 10, 1.0, 16, 17, 1.5, src_iso_cm=20.0, src_det_cm=36.0)
    orc = O.Oracle(g, S.default_spectra())
    N = 120
    M = np.zeros((16 * 17, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        M[:, k] = orc.project(e.reshape(10, 12)).ravel()
    y = np.random.default_rng(2).standard_normal((16, 17))
    np.testing.assert_allclose(orc.backproject(y).ravel(), M.T @ y.ravel(), rtol=1e-13,
                               atol=1e-13)
    assert np.count_nonzero(M) > 0


@pytest.mark.parametrize("kind", ["parallel", "fan"])
def test_adjointness(kind):
    if kind == "parallel":
        g = S.geometry("parallel", 64, 48, 0.5, 90, 95, 0.5, det_offset=0.25)
    else:
        g = S.fan_geometry_fov(64, 120, 160, fov_cm=25.6)
    orc = O.Oracle(g, S.default_spectra())
    rng = np.random.default_rng(3)
    x = rng.standard_normal((g["ny"], g["nx"]))
    y = rng.standard_normal((g["n_views"], g["n_det"]))
    Rx, RTy = orc.project(x), orc.backproject(y)
    lhs, rhs = float(np.sum(Rx * y)), float(np.sum(x * RTy))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Rx) * np.linalg.norm(y)


def test_finite_differences_and_transpose():
    ny, nx = 5, 7
    x = _linear_image(nx, ny, (1.0, 0.5, -2.0))
    Dx = O.D(x)
    np.testing.assert_array_equal(Dx[0][:, :-1], 0.5)
    np.testing.assert_array_equal(Dx[0][:, -1], 0.0)
    np.testing.assert_array_equal(Dx[1][:-1, :], -2.0)
    np.testing.assert_array_equal(Dx[1][-1, :], 0.0)
    # D^T equals the transpose of the explicit matrix of D.
    M = np.zeros((2 * ny * nx, ny * nx))
    for k in range(ny * nx):
        e = np.zeros(ny * nx)
        e[k] = 1.0
        M[:, k] = O.D(e.reshape(ny, nx)).ravel()
    yv = np.random.default_rng(4).standard_normal((2, ny, nx))
    np.testing.assert_allclose(O.DT(yv).ravel(), M.T @ yv.ravel(), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("v", [-3.0, -0.2, -0.05, 0.0, 0.04, 0.1, 2.5])
def test_shrinkage_is_prox_of_abs(v):
    t = 0.1
    res = minimize_scalar(lambda y: t * abs(y) + 0.5 * (y - v) ** 2, bounds=(-10, 10),
                          method="bounded", options=dict(xatol=1e-12))
    assert O.shrink(np.array([v]), t)[0] == pytest.approx(res.x, abs=1e-8)


def test_nonnegativity_projection():
    w = np.array([-2.0, -1e-9, 0.0, 3e-7, 4.0])
    z = np.maximum(0.0, w)
    # Projection onto R+: nearest nonnegative point.
    for wi, zi in zip(w, z):
        cand = np.linspace(0, 5, 50001)
        assert abs(zi - cand[np.argmin((cand - wi) ** 2)]) <= 1e-4
