"""The range argument of the joint spectra evaluation, checked against the oracle's
forward model on the CPU: for a trial step d from a point a, each spectrum's base-2
log-sum-exp L(a) = -f(a) / ln 2 (Eq. (3)) at a + d lies between the first-order
prediction L(a) - grad f(a) . d / ln 2 (L is convex in a) and L(a) plus the largest
change of any exponent, max_k(-kc_k d_c - kp_k d_p) with kc, kp = f_KN, f_p / ln 2.
The decomposition kernels place their shared shift between these bounds."""
import numpy as np

import oracle as O
from paper_1905_00934_amd import synth as S


def test_log_sum_exp_bounds_bracket_the_trial_value():
    spec = S.default_spectra()
    g = S.geometry("parallel", 4, 4, 1.0, 8, 8, 1.0)
    orc = O.Oracle(g, spec)
    rng = np.random.default_rng(3)
    n = 4000
    ac = rng.uniform(-5.0, 400.0, n)
    ap = rng.uniform(-3.0, 100.0, n)
    dc = rng.normal(0.0, 20.0, n)
    dp = rng.normal(0.0, 5.0, n)
    fh, fl, gh, gl = orc.forward(ac, ap)
    qh, ql, _, _ = orc.forward(ac + dc, ap + dp)
    ln2 = np.log(2.0)
    used = (spec.s_high > 0) | (spec.s_low > 0)
    kc = spec.f_kn[used] / ln2
    kp = spec.f_p[used] / ln2
    up = np.max(-np.outer(dc, kc) - np.outer(dp, kp), axis=1)
    gaps = []
    for f, g_, q in ((fh, gh, qh), (fl, gl, ql)):
        L = -f / ln2
        Lq = -q / ln2
        lower = L - (g_[:, 0] * dc + g_[:, 1] * dp) / ln2
        upper = L + up
        tol = 1e-9 * (1.0 + np.abs(L) + np.abs(Lq))
        assert np.all(Lq >= lower - tol)
        assert np.all(Lq <= upper + tol)
        gaps.append(np.min(upper - Lq))
    # The bounds are not vacuous: the upper one is reached closely by some steps.
    assert min(gaps) < 1.0
