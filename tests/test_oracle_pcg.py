"""Pins of the oracle's preconditioned CG (Sec. 3.3: a high-pass (ramp) filter
applied by FFT as the preconditioner of the shift-invariant Eq. (12))."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1905_00934_amd import synth as S

from test_oracle_admm import _cg_setup, _dense, _micro


def test_pad_shape_is_power_of_two_at_least_twice():
    assert O.pad_shape(5, 3) == (16, 8)
    assert O.pad_shape(512, 512) == (1024, 1024)
    assert O.pad_shape(384, 384) == (1024, 1024)
    assert O.pad_shape(29, 37) == (64, 128)
    assert O.pad_shape(1, 1) == (2, 2)


def test_ramp_filter_closed_form():
    f = O.ramp_filter(16, 8)
    assert f.shape == (16, 8)
    assert f[0, 0] == 1.0 / 16                       # floor at w = 0
    assert f[0, 1] == pytest.approx(1.0 / 8, abs=0)  # |w| = 1/8 cycles per pixel
    assert f[1, 0] == 1.0 / 16                       # |w| = 1/16 = floor
    assert f[8, 4] == pytest.approx(math.sqrt(0.25 + 0.25), rel=1e-15)  # both Nyquist
    assert f[3, 2] == pytest.approx(math.hypot(3 / 16, 2 / 8), rel=1e-15)
    # Even in frequency (a real symmetric kernel).
    for ky in range(16):
        for kx in range(8):
            assert f[ky, kx] == f[(-ky) % 16, (-kx) % 8]


def test_precondition_equals_direct_convolution():
    """M r written from the definitions: the kernel is the inverse DFT of the filter
    (summed term by term) and M r its linear convolution with r, cropped."""
    rng = np.random.default_rng(0)
    ny, nx = 5, 3
    r = rng.standard_normal((ny, nx))
    py, px = O.pad_shape(ny, nx)
    f = O.ramp_filter(py, px)
    h = np.zeros((py, px))
    for dy in range(py):
        for dx in range(px):
            acc = 0.0
            for ky in range(py):
                for kx in range(px):
                    acc += f[ky, kx] * math.cos(2 * math.pi * (ky * dy / py + kx * dx / px))
            h[dy, dx] = acc / (py * px)
    want = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            for jj in range(ny):
                for ii in range(nx):
                    want[j, i] += h[(j - jj) % py, (i - ii) % px] * r[jj, ii]
    np.testing.assert_allclose(O.precondition(r, f), want, rtol=1e-12, atol=1e-14)


def test_preconditioner_is_symmetric_positive_definite():
    ny, nx = 6, 5
    f = O.ramp_filter(*O.pad_shape(ny, nx))
    N = ny * nx
    M = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        M[:, k] = O.precondition(e.reshape(ny, nx), f).ravel()
    np.testing.assert_allclose(M, M.T, atol=1e-15)
    assert np.linalg.eigvalsh(M).min() > 0


def _dense_precond(shape):
    ny, nx = shape
    f = O.ramp_filter(*O.pad_shape(ny, nx))
    N = ny * nx
    M = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        M[:, k] = O.precondition(e.reshape(ny, nx), f).ravel()
    return f, M


def test_pcg_full_equals_dense_solve():
    orc, A, b, t, h, x0 = _cg_setup()
    f, _ = _dense_precond(orc.img_shape)
    x, Rx = orc.cg(x0, orc.project(x0), t, h, 30, filt=f)
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(A, b), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(Rx, orc.project(x), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_pcg_iterate_is_preconditioned_krylov_minimiser(n):
    """After n steps, PCG minimises the A-norm error over x0 + K_n(M A, M r0)."""
    orc, A, b, t, h, x0 = _cg_setup(seed=n + 10)
    f, M = _dense_precond(orc.img_shape)
    x, _ = orc.cg(x0, orc.project(x0), t, h, n, filt=f)
    r0 = b - A @ x0.ravel()
    K = np.stack([np.linalg.matrix_power(M @ A, k) @ (M @ r0) for k in range(n)], axis=1)
    Q, _ = np.linalg.qr(K)
    c = np.linalg.solve(Q.T @ A @ Q, Q.T @ r0)
    np.testing.assert_allclose(x.ravel(), x0.ravel() + Q @ c, rtol=1e-10, atol=1e-10)
    # One preconditioned step differs from one plain step (the filter is not flat).
    xc, _ = orc.cg(x0, orc.project(x0), t, h, n)
    assert np.linalg.norm(x - xc) > 1e-6 * np.linalg.norm(x)


def test_flat_filter_gives_plain_cg():
    orc, A, b, t, h, x0 = _cg_setup(seed=7)
    ones = np.ones(O.pad_shape(*orc.img_shape))
    xa, _ = orc.cg(x0, orc.project(x0), t, h, 3, filt=ones)
    xb, _ = orc.cg(x0, orc.project(x0), t, h, 3)
    np.testing.assert_allclose(xa, xb, rtol=1e-12, atol=1e-13)


def test_pcg_admm_x_step_is_exact_with_enough_iterations():
    """With as many PCG steps as pixels the x-update solves Eq. (12) exactly, so the
    x-step optimality R^T u^a + D^T u^y + u^z = R^T da + D^T dy + dz holds."""
    pr, orc, (mh, ml, wh, wl) = _micro()
    prm = O.Params(lam=(4e-2, 2e-2), rho0=(5.0, 10.0), lm_iters=20, cg_iters=64,
                   rho_mode="fixed", precond="ramp")
    st = orc.admm_init(mh, ml, wh, wl, prm)
    for _ in range(3):
        prev = st
        st = orc.admm_iterate(st, mh, ml, wh, wl, prm, 1)
        for b in range(2):
            lhs = orc.backproject(st.ua[b], count="RT_dual") + O.DT(st.uy[b]) + st.uz[b]
            rhs = (orc.backproject(st.a[b] - prev.a[b], count="RT_dual")
                   + O.DT(st.y[b] - prev.y[b]) + st.z[b] - prev.z[b])
            np.testing.assert_allclose(lhs, rhs, atol=1e-7 * (np.abs(rhs).max() + 1.0))
    with pytest.raises(ValueError):
        orc.admm_iterate(st, mh, ml, wh, wl, O.Params(precond="bogus"), 1)
