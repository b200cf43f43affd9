"""Pins of the oracle's CG x-update (Eq. (12)) and ADMM iteration (Eq. (9)-(13), Table 1)."""
import os

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from paper_1905_00934_amd import synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _micro(spec=None, noise=True, seed=3):
    g = S.geometry("parallel", 8, 8, 1.0, 24, 13, 1.0)
    ph = S.Phantom([S.Shape("ellipse", 0.3, -0.2, 2.5, 1.8, 0.4, 0.3, 0.02),
                    S.Shape("rect", -1.0, 1.2, 0.8, 0.6, 0.2, 1.0, 2.0)])
    pr = S.make_problem("micro", g, ph, 1e5, seed, spec=spec, noise=noise)
    orc = O.Oracle(g, pr.spec)
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    return pr, orc, (mh, ml, wh, wl)


def _dense(orc):
    ny, nx = orc.img_shape
    N = ny * nx
    M = np.zeros((orc.sino_shape[0] * orc.sino_shape[1], N))
    Dm = np.zeros((2 * N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        M[:, k] = orc.project(e.reshape(ny, nx), count=None).ravel()
        Dm[:, k] = O.D(e.reshape(ny, nx)).ravel()
    return M, Dm


def _cg_setup(seed=0):
    g = S.geometry("fan", 6, 5, 1.0, 10, 9, 1.6, src_iso_cm=15.0, src_det_cm=27.0)
    orc = O.Oracle(g, S.default_spectra())
    M, Dm = _dense(orc)
    A = M.T @ M + Dm.T @ Dm + np.eye(30)
    rng = np.random.default_rng(seed)
    t = rng.standard_normal(orc.sino_shape)
    h = rng.standard_normal(orc.img_shape)
    b = M.T @ t.ravel() + h.ravel()
    x0 = rng.standard_normal(orc.img_shape)
    return orc, A, b, t, h, x0


def test_cg_full_krylov_equals_dense_solve():
    orc, A, b, t, h, x0 = _cg_setup()
    x, Rx = orc.cg(x0, orc.project(x0), t, h, 30)
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(A, b), rtol=1e-9, atol=1e-9)
    # The tracked R x stays equal to R applied to the iterate.
    np.testing.assert_allclose(Rx, orc.project(x), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_cg_iterate_is_krylov_subspace_minimiser(n):
    """After n steps from x0, CG minimises the A-norm error over x0 + K_n(A, r0)."""
    orc, A, b, t, h, x0 = _cg_setup(seed=n)
    x, _ = orc.cg(x0, orc.project(x0), t, h, n)
    r0 = b - A @ x0.ravel()
    K = np.stack([np.linalg.matrix_power(A, k) @ r0 for k in range(n)], axis=1)
    Q, _ = np.linalg.qr(K)
    c = np.linalg.solve(Q.T @ A @ Q, Q.T @ r0)
    want = x0.ravel() + Q @ c
    np.testing.assert_allclose(x.ravel(), want, rtol=1e-10, atol=1e-10)


def test_table1_operator_counts():
    rows = [list(map(int, line.split())) for line in open(os.path.join(GOLDEN,
            "table1_operator_counts.txt")) if line.strip() and not line.startswith("#")]
    pr, orc, (mh, ml, wh, wl) = _micro()
    for m, n, nR, nRT, nf in rows:
        prm = O.Params(lm_iters=m, cg_iters=n, rho_mode="fixed")
        st = orc.admm_init(mh, ml, wh, wl, prm)
        for _ in range(2):
            before = dict(orc.counts)
            st = orc.admm_iterate(st, mh, ml, wh, wl, prm, 1)
            d = {k: orc.counts[k] - before[k] for k in orc.counts}
            assert d["R"] == nR and d["RT"] == nRT and d["RT_dual"] == 0
            # f and its gradient are evaluated together, so current-point evaluations
            # are reused: no more than the table's 4m per ray, and exactly 4m at m = 1.
            assert d["f"] <= nf and (m != 1 or d["f"] == nf)


def _grad_F(orc, a, mh, ml, wh, wl):
    fh, fl, gh, gl = orc.forward(a[0], a[1])
    rh, rl = wh * (fh - mh), wl * (fl - ml)
    return np.stack([rh * gh[..., 0] + rl * gl[..., 0], rh * gh[..., 1] + rl * gl[..., 1]])


@pytest.mark.parametrize("mode", ["fixed", "adaptive"])
def test_admm_subproblem_optimality_invariants(mode):
    """With exact sub-solves, after every iteration (for the rho then in force):
    a-step:  rho u^a = -grad F(a)                       (Eq. (13) optimality + Eq. (11))
    y-step:  |rho u^y| <= lambda, = -lambda sign(y) where y != 0   (Eq. (9))
    z-step:  z >= 0, u^z >= 0, z u^z = 0                (Eq. (10))
    x-step:  R^T u^a + D^T u^y + u^z = R^T da + D^T dy + dz   (Eq. (12) optimality)
    and the rho update rescales u so that rho u is unchanged."""
    pr, orc, (mh, ml, wh, wl) = _micro()
    lam = (4e-2, 2e-2)
    prm = O.Params(lam=lam, rho0=(5.0, 10.0), lm_iters=200, cg_iters=64, rho_mode=mode)
    st = orc.admm_init(mh, ml, wh, wl, prm)
    for it in range(12):
        prev = st
        st = orc.admm_iterate(st, mh, ml, wh, wl, prm, 1)
        rho = st.rho
        gF = _grad_F(orc, st.a, mh, ml, wh, wl)
        for b in range(2):
            # LM converges only linearly on large-residual rays, so the a-step optimality
            # holds to a small relative error overall (a sign or ordering mistake in the
            # a-step or the dual update gives an O(1) error here).
            assert (np.linalg.norm(rho[b] * st.ua[b] + gF[b])
                    <= 1e-2 * np.linalg.norm(gF[b]))
            ruy = rho[b] * st.uy[b]
            assert np.all(np.abs(ruy) <= lam[b] * (1 + 1e-9))
            nz = np.abs(st.y[b]) > 0
            np.testing.assert_allclose(ruy[nz], -lam[b] * np.sign(st.y[b][nz]), rtol=1e-9)
            assert np.all(st.z[b] >= 0) and np.all(st.uz[b] >= -1e-15)
            assert np.all(np.abs(st.z[b] * st.uz[b]) <= 1e-15)  # complementarity up to rounding
            # u was rescaled by rho_old / rho_new after the dual step.
            lhs = (orc.backproject(st.ua[b], count="RT_dual") + O.DT(st.uy[b])
                   + st.uz[b]) * (rho[b] / prev.rho[b])
            rhs = (orc.backproject(st.a[b] - prev.a[b], count="RT_dual")
                   + O.DT(st.y[b] - prev.y[b]) + st.z[b] - prev.z[b])
            np.testing.assert_allclose(lhs, rhs, atol=1e-7 * (np.abs(rhs).max() + 1.0))
    if mode == "adaptive":
        assert any(np.any(e["rho"] != prm.rho0) for e in st.log)


def test_admm_converges_to_direct_map_minimiser_without_tv():
    """Monochromatic data make Eq. (4) convex; with lambda = 0 its minimiser over x >= 0
    is found independently by L-BFGS-B, and ADMM iterates approach it."""
    pr, orc, (mh, ml, wh, wl) = _micro(spec=S.monochromatic_spectra(80.0, 40.0))

    def obj(xv):
        x = xv.reshape(2, 8, 8)
        a = [orc.project(x[0], count=None), orc.project(x[1], count=None)]
        fh, fl, gh, gl = orc.forward(a[0], a[1])
        rh, rl = wh * (fh - mh), wl * (fl - ml)
        val = 0.5 * (np.sum(wh * (fh - mh) ** 2) + np.sum(wl * (fl - ml) ** 2))
        gc = orc.backproject(rh * gh[..., 0] + rl * gl[..., 0])
        gp = orc.backproject(rh * gh[..., 1] + rl * gl[..., 1])
        return val, np.concatenate([gc.ravel(), gp.ravel()])

    res = minimize(obj, np.full(128, 0.05), jac=True, method="L-BFGS-B",
                   bounds=[(0, None)] * 128,
                   options=dict(maxiter=20000, ftol=1e-16, gtol=1e-12, maxfun=50000))
    xs = res.x.reshape(2, 8, 8)
    prm = O.Params(lam=(0.0, 0.0), rho0=(2.0, 2.0), lm_iters=20, cg_iters=128, rho_mode="fixed")
    st = orc.admm_init(mh, ml, wh, wl, prm)
    errs = []
    for _ in range(3):
        st = orc.admm_iterate(st, mh, ml, wh, wl, prm, 100)
        errs.append([np.linalg.norm(st.x[b] - xs[b]) / np.linalg.norm(xs[b]) for b in range(2)])
    errs = np.array(errs)
    assert np.all(np.diff(errs, axis=0) < 0)
    assert errs[-1, 0] < 0.02 and errs[-1, 1] < 0.15
    fx = orc.map_objective(st.x, mh, ml, wh, wl, (0.0, 0.0))
    assert res.fun <= fx <= res.fun * 1.01


def test_tiny_config_objective_and_residual_decrease():
    pr = S.tiny_problem(0)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    prm = O.Params()
    st = orc.admm_init(mh, ml, wh, wl, prm)
    f0 = orc.map_objective(st.x, mh, ml, wh, wl, prm.lam)
    st5 = orc.admm_iterate(st, mh, ml, wh, wl, prm, 5)
    st20 = orc.admm_iterate(st5, mh, ml, wh, wl, prm, 15)
    f5 = orc.map_objective(st5.x, mh, ml, wh, wl, prm.lam)
    f20 = orc.map_objective(st20.x, mh, ml, wh, wl, prm.lam)
    assert f20 < f5 < f0
    r1 = np.linalg.norm(st20.log[0]["r"])
    r20 = np.linalg.norm(st20.log[-1]["r"])
    assert r20 < r1
    # The Compton image moves toward the ground truth (Eq. (14)).
    assert O.xi_db(st20.x[0], pr.x_true[0]) < O.xi_db(st5.x[0], pr.x_true[0]) < 0
