"""Pins of the oracle's LM(m) x CG(n) baseline (Eqs. (7)-(8), Table 1)."""
import os

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from paper_1905_00934_amd import synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _micro(spec=None, seed=3):
    g = S.geometry("parallel", 8, 8, 1.0, 24, 13, 1.0)
    ph = S.Phantom([S.Shape("ellipse", 0.3, -0.2, 2.5, 1.8, 0.4, 0.3, 0.02),
                    S.Shape("rect", -1.0, 1.2, 0.8, 0.6, 0.2, 1.0, 2.0)])
    pr = S.make_problem("micro", g, ph, 1e5, seed, spec=spec)
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


def _start(orc, rng):
    """A nonzero start so that the rho terms of Eqs. (7)-(8) see y, z and u."""
    ny, nx = orc.img_shape
    x0 = np.stack([0.2 + 0.05 * rng.random((ny, nx)), 0.01 + 0.01 * rng.random((ny, nx))])
    return x0


def test_table1_operator_counts():
    rows = [list(map(int, line.split())) for line in open(os.path.join(
        GOLDEN, "table1_lmcg_operator_counts.txt")) if line.strip() and not line.startswith("#")]
    pr, orc, (mh, ml, wh, wl) = _micro()
    for m, n, nR, nRT, nf in rows:
        prm = O.Params(lm_iters=m, cg_iters=n, rho_mode="adaptive")
        st = orc.lmcg_init(mh, ml, wh, wl, prm)
        for _ in range(2):
            before = dict(orc.counts)
            st = orc.lmcg_iterate(st, mh, ml, wh, wl, prm, 1)
            d = {k: orc.counts[k] - before[k] for k in orc.counts}
            assert (d["R"], d["RT"], d["RT_dual"], d["f"]) == (nR, nRT, 0, nf)


def _phi_linear_solve(M, Dm, w, k_b, k_o, m, x_o, y, uy, z, uz, rho):
    """Minimiser of sum_s 1/2 ||w_s^1/2 (k_bs M x + k_os M x_o - m_s)||^2
    + rho/2 (||y - Dm x + uy||^2 + ||z - x + uz||^2), by a dense solve."""
    N = M.shape[1]
    A = rho * (Dm.T @ Dm + np.eye(N))
    rhs = rho * (Dm.T @ (y + uy) + z + uz)
    for s in range(2):
        Ws = np.diag(w[s])
        A += k_b[s] ** 2 * M.T @ Ws @ M
        rhs += k_b[s] * M.T @ Ws @ (m[s] - k_o[s] * (M @ x_o))
    return np.linalg.solve(A, rhs)


def test_monochromatic_undamped_step_is_the_exact_subproblem_minimiser():
    """With monochromatic spectra f is linear, so Eq. (7) is a quadratic in x_c; one
    undamped LM iteration with n = N CG steps lands on its minimiser, and Eq. (8)'s with
    the new x_c; both are found here by dense solves built from unit projections."""
    spec = S.monochromatic_spectra(80.0, 40.0)
    pr, orc, (mh, ml, wh, wl) = _micro(spec=spec)
    M, Dm = _dense(orc)
    rho = (0.7, 1.3)
    prm = O.Params(lm_iters=1, cg_iters=64, rho0=rho, lm_mu0=0.0, rho_mode="fixed",
                   lam=(0.0, 0.0))
    x0 = _start(orc, np.random.default_rng(1))
    st0 = orc.lmcg_init(mh, ml, wh, wl, prm, x0=x0)
    st = orc.lmcg_iterate(st0, mh, ml, wh, wl, prm, 1)
    # f_s(a) = f_KN(E_s) a_c + f_p(E_s) a_p at the single energy of each spectrum.
    fh, fl, gh, gl = orc.forward(np.zeros(1), np.zeros(1))
    kc, kp = (gh[0, 0], gl[0, 0]), (gh[0, 1], gl[0, 1])
    w = (wh.ravel(), wl.ravel())
    m = (mh.ravel(), ml.ravel())
    yv = [st0.y[b].ravel() for b in range(2)]
    xc = _phi_linear_solve(M, Dm, w, kc, kp, m, x0[1].ravel(), yv[0], 0 * yv[0],
                           x0[0].ravel(), 0 * yv[0][:64], rho[0])
    np.testing.assert_allclose(st.x[0].ravel(), xc, rtol=1e-8, atol=1e-10)
    xp = _phi_linear_solve(M, Dm, w, kp, kc, m, xc, yv[1], 0 * yv[1], x0[1].ravel(),
                           0 * yv[1][:64], rho[1])
    np.testing.assert_allclose(st.x[1].ravel(), xp, rtol=1e-8, atol=1e-10)
    # R x is the projection of the accepted image.
    np.testing.assert_allclose(st.Rx[0], orc.project(st.x[0], count=None), rtol=1e-12, atol=1e-12)


def test_monochromatic_damped_step_solves_the_shifted_system():
    """With damping, the step d solves (H + mu kappa I) d = -g, kappa = g'Hg / g'g."""
    spec = S.monochromatic_spectra(80.0, 40.0)
    pr, orc, (mh, ml, wh, wl) = _micro(spec=spec)
    M, Dm = _dense(orc)
    rho, mu = 0.9, 0.3
    prm = O.Params(lm_iters=1, cg_iters=64, rho0=(rho, rho), lm_mu0=mu, rho_mode="fixed",
                   lam=(0.0, 0.0))
    x0 = _start(orc, np.random.default_rng(2))
    st0 = orc.lmcg_init(mh, ml, wh, wl, prm, x0=x0)
    st = orc.lmcg_iterate(st0, mh, ml, wh, wl, prm, 1)
    fh, fl, gh, gl = orc.forward(np.zeros(1), np.zeros(1))
    kc, kp = (gh[0, 0], gl[0, 0]), (gh[0, 1], gl[0, 1])
    N = 64
    k = (kc, kp)

    def step(b, a):
        """Damped step of basis b at the projections a = (a_c, a_p); y = D x0, z = x0, u = 0."""
        xb = x0[b].ravel()
        H = rho * (Dm.T @ Dm + np.eye(N))
        g = rho * (Dm.T @ Dm @ xb + xb - Dm.T @ st0.y[b].ravel() - xb)
        for s, (ww, mm) in enumerate(((wh.ravel(), mh.ravel()), (wl.ravel(), ml.ravel()))):
            H += k[b][s] ** 2 * M.T @ np.diag(ww) @ M
            g += k[b][s] * M.T @ (ww * (kc[s] * a[0] + kp[s] * a[1] - mm))
        kappa = g @ H @ g / (g @ g)
        return np.linalg.solve(H + mu * kappa * np.eye(N), -g)

    xc = x0[0].ravel() + step(0, (M @ x0[0].ravel(), M @ x0[1].ravel()))
    np.testing.assert_allclose(st.x[0].ravel(), xc, rtol=1e-8, atol=1e-10)
    # Eq. (8) at the new x_c, with the damping restarted at mu0.
    xp = x0[1].ravel() + step(1, (M @ xc, M @ x0[1].ravel()))
    np.testing.assert_allclose(st.x[1].ravel(), xp, rtol=1e-8, atol=1e-10)


def test_polychromatic_lm_reaches_the_subproblem_minimiser():
    """Many LM iterations with full CG solve Eq. (7) on polychromatic data; its minimiser
    is found independently by L-BFGS-B on the objective written out here."""
    pr, orc, (mh, ml, wh, wl) = _micro()
    rho = 0.5
    x0 = _start(orc, np.random.default_rng(4))
    prm = O.Params(lm_iters=40, cg_iters=64, rho0=(rho, rho), rho_mode="fixed", lam=(0.0, 0.0))
    st0 = orc.lmcg_init(mh, ml, wh, wl, prm, x0=x0)
    y, z = st0.y[0], st0.z[0]
    ap = orc.project(x0[1], count=None)

    def obj(xv):
        x = xv.reshape(8, 8)
        ac = orc.project(x, count=None)
        fh, fl, gh, gl = orc.forward(ac, ap)
        eh, el = fh - mh, fl - ml
        dy = y - O.D(x)
        dz = z - x
        val = 0.5 * (np.sum(wh * eh ** 2) + np.sum(wl * el ** 2)) \
            + 0.5 * rho * (np.sum(dy ** 2) + np.sum(dz ** 2))
        grad = orc.backproject(wh * eh * gh[..., 0] + wl * el * gl[..., 0], count="RT_dual") \
            - rho * (O.DT(dy) + dz)
        return val, grad.ravel()

    res = minimize(obj, x0[0].ravel(), jac=True, method="L-BFGS-B",
                   options=dict(maxiter=20000, ftol=1e-16, gtol=1e-12, maxfun=50000))
    st = orc._lm_basis(st0.copy(), 0, mh, ml, wh, wl, rho, prm)
    np.testing.assert_allclose(st.x[0].ravel(), res.x, rtol=1e-5, atol=1e-7)
    # Steps are accepted only when they lower the objective.
    assert obj(st.x[0].ravel())[0] <= obj(x0[0].ravel())[0]


def test_lmcg_admm_converges_to_direct_map_minimiser_without_tv():
    """Eqs. (7)-(11) solve the same problem as the proposed splitting: with monochromatic
    data and lambda = 0 the LM x CG iterates approach the L-BFGS-B minimiser of Eq. (4)
    over x >= 0."""
    pr, orc, (mh, ml, wh, wl) = _micro(spec=S.monochromatic_spectra(80.0, 40.0))

    def obj(xv):
        x = xv.reshape(2, 8, 8)
        a = [orc.project(x[0], count=None), orc.project(x[1], count=None)]
        fh, fl, gh, gl = orc.forward(a[0], a[1])
        rh, rl = wh * (fh - mh), wl * (fl - ml)
        val = 0.5 * (np.sum(wh * (fh - mh) ** 2) + np.sum(wl * (fl - ml) ** 2))
        gc = orc.backproject(rh * gh[..., 0] + rl * gl[..., 0], count="RT_dual")
        gp = orc.backproject(rh * gh[..., 1] + rl * gl[..., 1], count="RT_dual")
        return val, np.concatenate([gc.ravel(), gp.ravel()])

    res = minimize(obj, np.full(128, 0.05), jac=True, method="L-BFGS-B",
                   bounds=[(0, None)] * 128,
                   options=dict(maxiter=20000, ftol=1e-16, gtol=1e-12, maxfun=50000))
    xs = res.x.reshape(2, 8, 8)
    prm = O.Params(lam=(0.0, 0.0), rho0=(2.0, 2.0), lm_iters=1, cg_iters=64, rho_mode="fixed")
    st = orc.lmcg_init(mh, ml, wh, wl, prm)
    errs = []
    for _ in range(4):
        st = orc.lmcg_iterate(st, mh, ml, wh, wl, prm, 60)
        errs.append([np.linalg.norm(st.x[b] - xs[b]) / np.linalg.norm(xs[b]) for b in range(2)])
    errs = np.array(errs)
    assert np.all(np.diff(errs, axis=0) < 0)
    assert errs[-1, 0] < 0.02 and errs[-1, 1] < 0.15
    fx = orc.map_objective(st.x, mh, ml, wh, wl, (0.0, 0.0))
    assert res.fun <= fx <= res.fun * 1.01


@pytest.mark.parametrize("mode", ["fixed", "adaptive"])
def test_lmcg_dual_step_invariants(mode):
    """After every iteration (for the rho then in force): |rho u^y| <= lambda with
    -lambda sign(y) where y != 0 (Eq. (9)); z >= 0, u^z >= 0, z u^z = 0 (Eq. (10)); the
    residual r = ||[y; z] - [D; I] x|| and rho balancing as logged."""
    pr, orc, (mh, ml, wh, wl) = _micro()
    lam = (4e-2, 2e-2)
    prm = O.Params(lam=lam, rho0=(5.0, 10.0), lm_iters=2, cg_iters=8, rho_mode=mode)
    st = orc.lmcg_init(mh, ml, wh, wl, prm)
    for _ in range(8):
        prev = st
        st = orc.lmcg_iterate(st, mh, ml, wh, wl, prm, 1)
        for b in range(2):
            ruy = st.rho[b] * st.uy[b]
            assert np.all(np.abs(ruy) <= lam[b] * (1 + 1e-9))
            nz = np.abs(st.y[b]) > 0
            np.testing.assert_allclose(ruy[nz], -lam[b] * np.sign(st.y[b][nz]), rtol=1e-9)
            assert np.all(st.z[b] >= 0) and np.all(st.uz[b] >= -1e-15)
            assert np.all(np.abs(st.z[b] * st.uz[b]) <= 1e-15)
            r = np.sqrt(np.sum((st.y[b] - O.D(st.x[b])) ** 2) + np.sum((st.z[b] - st.x[b]) ** 2))
            assert st.log[-1]["r"][b] == pytest.approx(r, rel=1e-12)
        # The f cache is f at R x of the accepted images.
        fh, fl, _, _ = orc.forward(orc.project(st.x[0], count=None),
                                   orc.project(st.x[1], count=None))
        np.testing.assert_allclose(st.fh, fh, rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(st.fl, fl, rtol=1e-11, atol=1e-12)
    if mode == "adaptive":
        assert any(np.any(e["rho"] != prm.rho0) for e in st.log)


def test_tiny_config_lmcg_data_term_and_xi_improve():
    """Only the sub-objectives of Eqs. (7)-(8) must decrease; on the tiny config the data
    term falls and the Compton image moves toward the ground truth (Eq. (14))."""
    pr = S.tiny_problem(0)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    prm = O.Params()
    st = orc.lmcg_init(mh, ml, wh, wl, prm)
    d0 = orc.data_cost(st.Rx[0], st.Rx[1], mh, ml, wh, wl)
    st5 = orc.lmcg_iterate(st, mh, ml, wh, wl, prm, 5)
    st15 = orc.lmcg_iterate(st5, mh, ml, wh, wl, prm, 10)
    assert st15.log[-1]["data"] < st5.log[-1]["data"] < d0
    assert st5.log[-1]["data"] == pytest.approx(
        orc.data_cost(st5.Rx[0], st5.Rx[1], mh, ml, wh, wl), rel=1e-12)
    assert O.xi_db(st15.x[0], pr.x_true[0]) < O.xi_db(st5.x[0], pr.x_true[0]) < 0
