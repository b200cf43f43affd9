"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Tolerances: FP64 operators agree with the oracle to rounding (1e-12 relative);
FP32 projections to 1e-5 relative L2 per view; after a fixed number of ADMM
iterations x_c within 1e-3 and x_p within 5e-3 (relative L2).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_1905_00934_amd import synth as S

pytestmark = pytest.mark.gpu

F64, F32 = torch.float64, torch.float32


@pytest.fixture(scope="module")
def dect():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00934_amd import dect as D
    D.lib()
    return D


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


GEOMS = {
    "tiny_parallel": S.geometry("parallel", 64, 64, 0.5, 90, 95, 0.5),
    "ragged_fan": S.geometry("fan", 37, 29, 0.4, 50, 71, 0.45, det_offset=0.3,
                             src_iso_cm=30.0, src_det_cm=52.0, angle0=0.1),
    "ragged_parallel": S.geometry("parallel", 33, 47, 0.5, 41, 300, 0.17, det_offset=-0.25,
                                  angle0=0.05),
    "single_view_fan": S.geometry("fan", 16, 16, 1.0, 1, 257, 0.3, src_iso_cm=40.0,
                                  src_det_cm=70.0),
    "two_by_two": S.geometry("parallel", 2, 2, 1.0, 7, 5, 0.8),
    # Full-turn fans with n_views % 4 == 0 on square images use the quarter-turn
    # symmetric operator (views v + k V/4 are rotations of base views).
    "sym_fan": S.fan_geometry_fov(64, 120, 100, fov_cm=25.6, src_iso_cm=40.0, src_det_cm=70.0),
    "sym_fan_offset": S.geometry("fan", 32, 32, 0.5, 44, 57, 0.6, det_offset=0.37,
                                 src_iso_cm=30.0, src_det_cm=50.0, angle0=0.2),
}


@pytest.mark.parametrize("gname", list(GEOMS))
@pytest.mark.parametrize("ch", [1, 2, 4])
def test_project_and_backproject_fp64_match_oracle(dect, gname, ch):
    g = GEOMS[gname]
    spec = S.default_spectra()
    orc = O.Oracle(g, spec)
    plan = dect.Plan(g, spec, F64)
    rng = np.random.default_rng(ch)
    img = rng.uniform(-1, 1, (g["ny"], g["nx"], ch))
    sino = rng.uniform(-1, 1, (g["n_views"], g["n_det"], ch))
    sq = (lambda a: a[..., 0]) if ch == 1 else (lambda a: a)
    Rg = host(plan.project(dev(sq(img), F64)))
    Bg = host(plan.backproject(dev(sq(sino), F64)))
    Rg = Rg.reshape(g["n_views"], g["n_det"], ch)
    Bg = Bg.reshape(g["ny"], g["nx"], ch)
    for c in range(ch):
        want_r = orc.project(img[..., c])
        want_b = orc.backproject(sino[..., c])
        assert np.max(np.abs(Rg[..., c] - want_r)) <= 1e-12 * max(np.abs(want_r).max(), 1.0)
        assert np.max(np.abs(Bg[..., c] - want_b)) <= 1e-12 * max(np.abs(want_b).max(), 1.0)
    # The GPU pair is an exact transpose up to summation order.
    lhs = float(np.sum(Rg * sino))
    rhs = float(np.sum(img * Bg))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Rg) * np.linalg.norm(sino)


@pytest.fixture(scope="module")
def slice512():
    return S.slice_problem(0, with_image=True)


def test_project_backproject_fp32_full_size(dect, slice512):
    pr = slice512
    orc = O.Oracle(pr.geom, pr.spec)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    img = np.stack(pr.x_true, -1)
    Rg = host(plan.project(dev(img, F32)))
    for c in range(2):
        want = orc.project(img[..., c])
        per_view = np.linalg.norm(Rg[..., c] - want, axis=1) / np.maximum(
            np.linalg.norm(want, axis=1), 1e-30)
        assert per_view.max() <= 1e-5, per_view.max()
    sino = np.stack(pr.a_true, -1)
    Bg = host(plan.backproject(dev(sino, F32)))
    for c in range(2):
        want = orc.backproject(sino[..., c])
        assert rel(Bg[..., c], want) <= 1e-5
    # Single-channel calls at full size and the 4-channel layout give the same numbers.
    R1 = host(plan.project(dev(img[..., 0], F32)))
    np.testing.assert_array_equal(R1, Rg[..., 0])
    img4 = np.concatenate([img, img[..., ::-1]], -1)
    R4 = host(plan.project(dev(img4, F32)))
    np.testing.assert_array_equal(R4[..., :2], Rg)


def _meas(pr):
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    return mh, ml, wh, wl


def test_ingest_matches_definition(dect):
    pr = S.tiny_problem(0)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    out = plan.ingest(dev(pr.counts_high, F64), dev(pr.counts_low, F64), pr.i0)
    for got, want in zip(out, _meas(pr)):
        np.testing.assert_allclose(host(got), want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("iters", [1, 3])
def test_decompose_fp64_matches_oracle(dect, iters):
    pr = S.tiny_problem(0)
    orc = O.Oracle(pr.geom, pr.spec)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    mh, ml, wh, wl = _meas(pr)
    rng = np.random.default_rng(5)
    ac0, ap0 = orc.linearised(mh, ml)
    vc = pr.a_true[0] + rng.normal(0, 0.05, mh.shape)
    vp = pr.a_true[1] + rng.normal(0, 0.05, mh.shape)
    rho = (1e-3, 3e-3)
    wc, wp, _ = orc.udm(mh, ml, wh, wl, vc, vp, rho[0], rho[1], iters, ac0, ap0)
    a = dev(np.stack([ac0, ap0], -1), F64)
    v = dev(np.stack([vc, vp], -1), F64)
    cost = torch.empty(mh.shape, dtype=F64, device="cuda")
    plan.decompose_rays(*(dev(m, F64) for m in (mh, ml, wh, wl)), a, v, rho, iters, cost)
    got = host(a)
    assert rel(got[..., 0], wc) <= 1e-10
    assert rel(got[..., 1], wp) <= 1e-10


def _wide_rays(orc, spec, n_views, n_det, seed):
    """Rays from air to metal: view row r holds line integrals up to (1000, 300) r / V,
    so whole 64-ray waves lie on either side of the distance in log-sum-exp at which the
    two spectra stop sharing one shift; noisy measurements, unit weights."""
    rng = np.random.default_rng(seed)
    t = (np.arange(n_views)[:, None] + rng.uniform(0, 1, (n_views, n_det))) / n_views
    ac = 1000.0 * t
    ap = 300.0 * t * rng.uniform(0.2, 1.0, t.shape)
    fh, fl, _, _ = orc.forward(ac, ap)
    mh = fh + rng.normal(0, 0.05, t.shape)
    ml = fl + rng.normal(0, 0.05, t.shape)
    return ac, ap, mh, ml


def _has_joint_table(spec):
    """Whether the plan evaluates the spectra together: every normalised weight is at least
    2^-24, so that with the shift at a spectrum's largest exponent no A_k overflows."""
    w = [s / s.sum() for s in (spec.s_high, spec.s_low)]
    return min(v[v > 0].min() for v in w) >= 2.0 ** -24


def _decompose_case(dect, spec, seed):
    g = S.geometry("parallel", 4, 4, 1.0, 16, 64, 1.0)
    orc = O.Oracle(g, spec)
    ac, ap, mh, ml = _wide_rays(orc, spec, 16, 64, seed)
    wh = np.ones_like(mh)
    wl = np.ones_like(ml)
    rng = np.random.default_rng(seed + 1)
    vc = ac + rng.normal(0, 0.5, ac.shape)
    vp = ap + rng.normal(0, 0.5, ap.shape)
    ac0, ap0 = orc.linearised(mh, ml)
    rho = (1e-3, 3e-3)
    want = orc.udm(mh, ml, wh, wl, vc, vp, rho[0], rho[1], 3, ac0, ap0)
    plan = dect.Plan(g, spec, F64)
    a = dev(np.stack([ac0, ap0], -1), F64)
    plan.decompose_rays(*(dev(m, F64) for m in (mh, ml, wh, wl)), a,
                        dev(np.stack([vc, vp], -1), F64), rho, 3)
    got = host(a)
    assert np.isfinite(got).all()
    assert rel(got[..., 0], want[0]) <= 1e-10
    assert rel(got[..., 1], want[1]) <= 1e-10
    return orc, want


def test_decompose_fp64_air_to_metal(dect):
    """Rays from air to metal: the two spectra's log-sum-exps lie up to ~175 (base 2)
    apart, and the first LM steps from the linearised start are long.  The shared shift
    of the joint evaluation and its per-spectrum fallback give the oracle's results."""
    spec = S.default_spectra()
    assert _has_joint_table(spec)
    orc, want = _decompose_case(dect, spec, 11)
    fh, fl, _, _ = orc.forward(want[0], want[1])
    assert (np.abs(fh - fl) / np.log(2)).max() > 100


def test_decompose_fp64_without_joint_table(dect):
    """A spectrum with a bin weighted below 2^-24 of its total leaves the plan without
    the joint evaluation (its inverse weight would take A_k out of range); the spectra
    are then evaluated apart, with the same results as the oracle."""
    base = S.default_spectra()
    s_high = base.s_high.copy()
    k = int(np.flatnonzero(s_high > 0)[-1])
    s_high[k] = 1e-40 * s_high.sum()
    spec = S.Spectra(base.energy_kev, s_high, base.s_low, base.f_kn, base.f_p)
    assert not _has_joint_table(spec)
    _decompose_case(dect, spec, 12)


def test_decompose_fp32_full_size(dect, slice512):
    pr = slice512
    orc = O.Oracle(pr.geom, pr.spec)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    mh, ml, wh, wl = _meas(pr)
    ac0, ap0 = orc.linearised(mh, ml)
    rng = np.random.default_rng(6)
    vc = pr.a_true[0] + rng.normal(0, 0.05, mh.shape)
    vp = pr.a_true[1] + rng.normal(0, 0.05, mh.shape)
    rho = (1e-3, 1e-3)
    wc, wp, _ = orc.udm(mh, ml, wh, wl, vc, vp, rho[0], rho[1], 2, ac0, ap0)
    a = dev(np.stack([ac0, ap0], -1), F32)
    plan.decompose_rays(*(dev(m, F32) for m in (mh, ml, wh, wl)), a,
                        dev(np.stack([vc, vp], -1), F32), rho, 2)
    got = host(a)
    assert rel(got[..., 0], wc) <= 1e-4
    assert rel(got[..., 1], wp) <= 1e-3
    # Rays where single precision took a different accept/reject branch are rare.
    far = np.abs(got[..., 0] - wc) > 1e-3 * (np.abs(wc) + 1)
    assert far.mean() < 1e-3


def test_decompose_fp32_noiseless_recovery(dect):
    spec = S.default_spectra()
    g = S.geometry("parallel", 4, 4, 1.0, 11, 13, 1.0)
    plan = dect.Plan(g, spec, F32)
    orc = O.Oracle(g, spec)
    gc, gp = np.meshgrid(np.linspace(0, 12, 13), np.linspace(0, 25, 11))
    ac_t, ap_t = gc, gp  # [11, 13]: one ray per (view, bin)
    lh, ll = S.expected_counts(spec, ac_t, ap_t, 1e5)
    mh, ml = -np.log(lh / 1e5), -np.log(ll / 1e5)
    a0 = np.stack(orc.linearised(mh, ml), -1)
    a = dev(a0, F32)
    plan.decompose_rays(*(dev(m, F32) for m in (mh, ml, lh / 1e5, ll / 1e5)), a, None,
                        (0.0, 0.0), 30)
    got = host(a)
    np.testing.assert_allclose(got[..., 0], ac_t, rtol=2e-4, atol=2e-4)
    np.testing.assert_allclose(got[..., 1], ap_t, rtol=2e-3, atol=2e-3)


def _admm_oracle(pr, prm, n):
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    st = orc.admm_init(mh, ml, wh, wl, prm)
    st = orc.admm_iterate(st, mh, ml, wh, wl, prm, n)
    return st


def _admm_gpu(dect, pr, dtype, params, n):
    plan = dect.Plan(pr.geom, pr.spec, dtype)
    meas = [dev(m, dtype) for m in _meas(pr)]
    st = plan.new_state()
    plan.admm_init(meas, st, params)
    log = plan.admm_iterate(meas, st, params, n, log=True)
    return plan, st, log


def test_admm_fp64_tiny_matches_oracle(dect):
    pr = S.tiny_problem(0)
    prm = O.Params()
    ost = _admm_oracle(pr, prm, 20)
    _, st, log = _admm_gpu(dect, pr, F64, dect.AdmmParams(), 20)
    x = host(st.x)
    for b in range(2):
        assert rel(x[..., b], ost.x[b]) <= 1e-8
    a = host(st.a)
    assert rel(a[..., 0], ost.a[0]) <= 1e-8
    assert [e["rho"] for e in log] == [tuple(e["rho"]) for e in ost.log]
    for eg, eo in zip(log, ost.log):
        np.testing.assert_allclose(eg["r"], eo["r"], rtol=1e-7)
        np.testing.assert_allclose(eg["s"], eo["s"], rtol=1e-7)
    _check_objective_log(log, ost.log)


def test_admm_fp64_without_joint_table_matches_oracle(dect):
    """The ADMM on a plan whose spectra are evaluated apart (a bin weighted below 2^-24 of
    its spectrum), as every decomposition kernel has both forms."""
    import types
    pr = S.tiny_problem(0)
    s_high = pr.spec.s_high.copy()
    s_high[int(np.flatnonzero(s_high > 0)[-1])] = 1e-40 * s_high.sum()
    spec = S.Spectra(pr.spec.energy_kev, s_high, pr.spec.s_low, pr.spec.f_kn, pr.spec.f_p)
    assert not _has_joint_table(spec)
    pr2 = types.SimpleNamespace(geom=pr.geom, spec=spec, counts_high=pr.counts_high,
                                counts_low=pr.counts_low, i0=pr.i0)
    prm = O.Params(cg_iters=2, lm_iters=2)
    ost = _admm_oracle(pr2, prm, 8)
    _, st, log = _admm_gpu(dect, pr2, F64, dect.AdmmParams(cg_iters=2, lm_iters=2), 8)
    x = host(st.x)
    for b in range(2):
        assert rel(x[..., b], ost.x[b]) <= 1e-8
    assert [e["rho"] for e in log] == [tuple(e["rho"]) for e in ost.log]
    _check_objective_log(log, ost.log)


def _check_objective_log(log, olog, rtol_data=1e-9, rtol_tv=1e-8):
    """The logged split objective (the serving stop criterion) against the oracle's:
    the data fit 1/2 sum w (f(a) - m)^2 at the new a and lambda |y|_1 at the new y,
    iteration by iteration."""
    assert len(log) == len(olog)
    for eg, eo in zip(log, olog):
        assert eg["flags"] == 0
        assert eg["data"] == pytest.approx(eo["data"], rel=rtol_data)
        assert eg["tv"] == pytest.approx(eo["tv"], rel=rtol_tv, abs=1e-14)
        assert eg["data"] + eg["tv"] == pytest.approx(eo["phi"], rel=rtol_data)


def test_admm_fp64_symmetric_fan_matches_oracle(dect):
    """Quarter-turn symmetric fan (the quad-record path of R and R^T) in FP64."""
    g = GEOMS["sym_fan"]
    k = g["nx"] * g["pixel_cm"] / 32.0
    ph = S.tiny_phantom(5)
    ph = S.Phantom([S.Shape(sh.kind, k * sh.cx, k * sh.cy, k * sh.ax, k * sh.ay, sh.rot,
                            sh.xc, sh.xp) for sh in ph.shapes])
    pr = S.make_problem("sym_fan", g, ph, 1e5, 5, with_image=False)
    prm = O.Params(cg_iters=2, lm_iters=2)
    ost = _admm_oracle(pr, prm, 8)
    _, st, log = _admm_gpu(dect, pr, F64, dect.AdmmParams(cg_iters=2, lm_iters=2), 8)
    x = host(st.x)
    for b in range(2):
        assert rel(x[..., b], ost.x[b]) <= 1e-8
    assert [e["rho"] for e in log] == [tuple(e["rho"]) for e in ost.log]
    _check_objective_log(log, ost.log)


@pytest.mark.parametrize("n, views, bins", [(48, 88, 80), (40, 72, 66)])
def test_admm_fp64_symmetric_fan_sizes_match_oracle(dect, n, views, bins):
    """CG(1) on quarter-turn symmetric fans whose right-hand side takes the other
    paths: n = 48 writes the orbit images with the right-hand side in plain tile order
    (9 quadrant tiles, not a multiple of the 8 XCDs), n = 40 (n % 16 != 0) runs the
    right-hand side and the orbit images as two kernels."""
    g = S.fan_geometry_fov(n, views, bins, fov_cm=0.4 * n, src_iso_cm=40.0, src_det_cm=70.0)
    k = g["nx"] * g["pixel_cm"] / 32.0
    ph = S.tiny_phantom(7)
    ph = S.Phantom([S.Shape(sh.kind, k * sh.cx, k * sh.cy, k * sh.ax, k * sh.ay, sh.rot,
                            sh.xc, sh.xp) for sh in ph.shapes])
    pr = S.make_problem(f"sym_fan{n}", g, ph, 1e5, 7, with_image=False)
    prm = O.Params()
    ost = _admm_oracle(pr, prm, 8)
    _, st, log = _admm_gpu(dect, pr, F64, dect.AdmmParams(), 8)
    x = host(st.x)
    for b in range(2):
        assert rel(x[..., b], ost.x[b]) <= 1e-8
    assert [e["rho"] for e in log] == [tuple(e["rho"]) for e in ost.log]
    _check_objective_log(log, ost.log)


# Problems of the FP32 parity runs: the uneven mix's 256^2 / 360 x 512 and
# 384^2 / 540 x 768 classes, and the single 512^2 / 720 x 1024 luggage slice.
FP32_CASES = {
    "fan256": lambda: S.uneven_problem(0, with_image=False),
    "fan384": lambda: S.uneven_problem(1, with_image=False),
    "fan512": lambda: S.slice_problem(0, with_image=False),
}

# A replayed single-precision decision that the oracle takes the other way, on a ray
# whose decomposition both sides start from the same point (within SAME_A, absolute plus
# relative), must be a near-tie.  LM accept test: |Phi(trial) - Phi(current)| within
# LM_TIE_MAX rounding scales (2^-23 times the first-order error bound of Phi, which
# includes the cancellation of f's log-sum-exp; the single-precision f carries besides
# the rounding of a ~110-term sum and the hardware exp2/log2, a few tens of such units
# at most).  Balancing test: r and mu s (or s and mu r) within RHO_TIE_MAX of each other,
# relative (the residual norms agree with the oracle's to ~1e-5 in single precision).
# The per-ray problem of Eq. (13) is not convex: where the two sides' starting points
# have drifted apart, LM may follow different local paths; such rays are counted, and at
# most SPLIT_MAX of them may end more than 1e-2 (absolute plus relative) apart.
LM_TIE_MAX = 512.0
RHO_TIE_MAX = 1e-3
SAME_A = 1e-4
SPLIT_MAX = 1e-3


def _fp32_lockstep(dect, pr, n_iters, pcg=False, rt_sums=0):
    """n_iters ADMM iterations of the FP32 library, one call each with its own adaptive rho,
    and of the oracle on the same single-precision inputs replaying, iteration by
    iteration, the library's LM accept decisions and rho choices (pcg: both with the ramp
    preconditioner).  Returns the oracle's state, the library's state and log, and the
    largest near-tie ratio of a replayed LM decision on a ray both sides started from the
    same point."""
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    meas64 = [r32(m) for m in _meas(pr)]
    orc = O.Oracle(pr.geom, pr.spec)
    prm = O.Params(precond="ramp" if pcg else None)
    ost = orc.admm_init(*meas64, prm)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    meas = [dev(m, F32) for m in meas64]
    params = dect.AdmmParams(precond=dect.PRECOND_RAMP if pcg else dect.PRECOND_NONE,
                             rt_sums=rt_sums)
    st = plan.new_state()
    plan.admm_init(meas, st, params)
    log, tie = [], 0.0
    for k in range(n_iters):
        a_lib = host(st.a)
        same = np.all(np.abs(a_lib - np.moveaxis(ost.a, 0, -1))
                      <= SAME_A * (1.0 + np.abs(a_lib)), axis=-1)
        log += plan.admm_iterate(meas, st, params, 1, log=True)
        bits = st.lm_accept.cpu().numpy().copy()
        rho_next = tuple(float(v) for v in st.scalars[:2].cpu().numpy())
        ost = orc.admm_iterate(ost, *meas64, prm, 1, lm_force=[bits], rho_force=[rho_next])
        tie = max(tie, float(np.max(np.where(same, ost.lm_ties, 0.0))))
    return ost, st, log, tie


@pytest.mark.parametrize("n_iters,case", [
    (3, "fan512"),
    (50, "fan256"),
    pytest.param(50, "fan384", marks=[pytest.mark.slow, pytest.mark.timeout(600)]),
    pytest.param(50, "fan512", marks=[pytest.mark.slow, pytest.mark.timeout(900)]),
])
def test_admm_fp32_matches_oracle_after_fixed_iterations(dect, n_iters, case):
    """FP32 fan-beam slices against the FP64 oracle after the configured 50 iterations (and
    3 at 512^2), x_c within 1e-3 and x_p within 5e-3.  The per-ray LM accept test and the
    residual-balancing test are discrete decisions taken in each side's precision; the
    oracle replays the library's, on the same single-precision inputs, and every one it
    would have taken the other way from the same starting point must be a near-tie at
    single precision.  The 384^2 class has 135 base views, an odd count, so the
    projector's last group of base views is partial."""
    pr = FP32_CASES[case]()
    print(f"\n[fp32 parity] {case} {pr.geom['nx']}^2 {pr.geom['n_views']}x{pr.geom['n_det']} "
          f"{n_iters} iterations in lockstep", flush=True)
    ost, st, log, tie = _fp32_lockstep(dect, pr, n_iters)
    x = host(st.x)
    a = host(st.a)
    flips = sum(e.get("lm_flips", 0) for e in ost.log)
    rtie = max(e.get("rho_tie", 0.0) for e in ost.log)
    split = float(np.mean(np.any(np.abs(a - np.moveaxis(ost.a, 0, -1))
                                 > 1e-2 * (1.0 + np.abs(a)), axis=-1)))
    ec, ep = rel(x[..., 0], ost.x[0]), rel(x[..., 1], ost.x[1])
    print(f"[fp32 parity] {case}: x_c {ec:.3e} x_p {ep:.3e}; replayed LM decisions the oracle "
          f"would have taken the other way: {flips}, largest near-tie ratio from a shared "
          f"start {tie:.3g}; rays ending apart {split:.2e}; rho tie {rtie:.3g}", flush=True)
    assert ec <= 1e-3
    assert ep <= 5e-3
    assert tie <= LM_TIE_MAX
    assert rtie <= RHO_TIE_MAX
    assert split <= SPLIT_MAX
    # The logged objective follows the oracle's: single-precision a and y change the
    # data fit and the TV term by far less than the x tolerance.
    _check_objective_log(log, ost.log, rtol_data=1e-3, rtol_tv=1e-3)
    assert [tuple(e["rho"]) for e in log] == [tuple(e["rho"]) for e in ost.log]


def test_admm_pcg_fp64_256_matches_oracle_after_50_iterations(dect):
    """UDM1-PCG1 (the ramp-preconditioned CG of the x-update, Sec. 3.3) on the 256^2
    fan slice in double precision: after 50 iterations, with the oracle replaying the
    library's LM decisions and rho choices (exact ties can fall either way), x_c and
    x_p agree to 1e-9."""
    pr = FP32_CASES["fan256"]()
    meas64 = list(_meas(pr))
    orc = O.Oracle(pr.geom, pr.spec)
    prm = O.Params(precond="ramp")
    ost = orc.admm_init(*meas64, prm)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    meas = [dev(m, F64) for m in meas64]
    params = dect.AdmmParams(precond=dect.PRECOND_RAMP)
    st = plan.new_state()
    plan.admm_init(meas, st, params)
    for _ in range(50):
        plan.admm_iterate(meas, st, params, 1)
        bits = st.lm_accept.cpu().numpy().copy()
        rho_next = tuple(float(v) for v in st.scalars[:2].cpu().numpy())
        ost = orc.admm_iterate(ost, *meas64, prm, 1, lm_force=[bits], rho_force=[rho_next])
    x = host(st.x)
    ec, ep = rel(x[..., 0], ost.x[0]), rel(x[..., 1], ost.x[1])
    print(f"\n[pcg fp64] fan256 50 iterations: x_c {ec:.3e} x_p {ep:.3e}", flush=True)
    assert ec <= 1e-9 and ep <= 1e-9


@pytest.mark.parametrize("case", [
    "fan256",
    pytest.param("fan512", marks=[pytest.mark.slow, pytest.mark.timeout(900)]),
])
def test_admm_pcg_fp32_matches_oracle_after_20_iterations(dect, case):
    """UDM1-PCG1 in single precision against the FP64 oracle in lockstep (as above),
    after 20 iterations: x_c within 1e-3 and x_p within 5e-3.  The preconditioned
    direction is ramp filtered, so the terms of R^T over its projection nearly cancel,
    and the single-precision sums of R^T lose enough digits that the iterates drift
    from the oracle by about 3e-5 per iteration in x_c (1.4e-3 after 50 iterations at
    256^2, where the double-precision library stays within 1e-11; 3.4e-4 with R^T
    summing in double), against 2e-6 with plain CG.  The near-tie check of the LM
    decisions is not applied: once the states differ by more than rounding, so do the
    inputs of a decision."""
    pr = FP32_CASES[case]()
    print(f"\n[pcg fp32] {case} 20 iterations in lockstep", flush=True)
    ost, st, log, tie = _fp32_lockstep(dect, pr, 20, pcg=True)
    x = host(st.x)
    ec, ep = rel(x[..., 0], ost.x[0]), rel(x[..., 1], ost.x[1])
    rtie = max(e.get("rho_tie", 0.0) for e in ost.log)
    print(f"[pcg fp32] {case}: x_c {ec:.3e} x_p {ep:.3e}; largest LM near-tie ratio {tie:.3g}; "
          f"rho tie {rtie:.3g}", flush=True)
    assert ec <= 1e-3
    assert ep <= 5e-3
    assert rtie <= RHO_TIE_MAX
    # The logged objective follows the oracle's, and the rho sequences are the same.
    _check_objective_log(log, ost.log, rtol_data=1e-3, rtol_tv=1e-3)
    assert [tuple(e["rho"]) for e in log] == [tuple(e["rho"]) for e in ost.log]


def test_admm_pcg_fp32_double_sums_match_oracle_after_50_iterations(dect):
    """UDM1-PCG1 on the FP32 plan with the transposes summing in double precision
    (dect_rt_sums F64) against the FP64 oracle in lockstep after 50 iterations at 256^2:
    x_c within 1e-3 and x_p within 5e-3, where single-precision sums drift past 1e-3."""
    pr = FP32_CASES["fan256"]()
    print("\n[pcg fp32, double sums] fan256 50 iterations in lockstep", flush=True)
    ost, st, log, tie = _fp32_lockstep(dect, pr, 50, pcg=True, rt_sums=dect.RT_SUMS_F64)
    x = host(st.x)
    ec, ep = rel(x[..., 0], ost.x[0]), rel(x[..., 1], ost.x[1])
    rtie = max(e.get("rho_tie", 0.0) for e in ost.log)
    print(f"[pcg fp32, double sums]: x_c {ec:.3e} x_p {ep:.3e}; rho tie {rtie:.3g}", flush=True)
    assert ec <= 1e-3
    assert ep <= 5e-3
    assert rtie <= RHO_TIE_MAX
    _check_objective_log(log, ost.log, rtol_data=1e-3, rtol_tv=1e-3)
    assert [tuple(e["rho"]) for e in log] == [tuple(e["rho"]) for e in ost.log]


def test_double_sums_leave_fp64_plans_unchanged(dect):
    """An FP64 plan sums in double either way: the option changes no bit of its state."""
    pr = S.tiny_problem(0)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    meas = [dev(m, F64) for m in _meas(pr)]
    states = []
    for sums in (dect.RT_SUMS_PLAN, dect.RT_SUMS_F64):
        prm = dect.AdmmParams(rt_sums=sums)
        st = plan.new_state()
        plan.admm_init(meas, st, prm)
        plan.admm_iterate(meas, st, prm, 5)
        states.append(st)
    torch.cuda.synchronize()
    assert torch.equal(states[0].buf, states[1].buf)
    with pytest.raises(dect.DectError):
        plan.admm_iterate(meas, states[0], dect.AdmmParams(rt_sums=2), 1)


def test_checkpoint_resume_and_determinism(dect):
    pr = S.tiny_problem(1)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    meas = [dev(m, F32) for m in _meas(pr)]
    params = dect.AdmmParams()
    s1 = plan.new_state()
    plan.admm_init(meas, s1, params)
    plan.admm_iterate(meas, s1, params, 20)
    s2 = plan.new_state()
    plan.admm_init(meas, s2, params)
    plan.admm_iterate(meas, s2, params, 10)
    saved = s2.buf.clone()
    s3 = plan.new_state()
    s3.buf.copy_(saved)
    plan.admm_iterate(meas, s3, params, 10)
    torch.cuda.synchronize()
    assert torch.equal(s1.x, s3.x) and torch.equal(s1.a, s3.a)
    assert torch.equal(s1.scalars[:4], s3.scalars[:4])


def test_errors_are_reported(dect):
    spec = S.default_spectra()
    with pytest.raises(dect.DectError, match="E_SHAPE"):
        dect.Plan(S.geometry("fan", 64, 64, 1.0, 10, 10, 1.0, src_iso_cm=30.0,
                             src_det_cm=50.0), spec, F32)
    plan = dect.Plan(GEOMS["ragged_fan"], spec, F32)
    img = torch.zeros((29, 37, 3), dtype=F32, device="cuda")
    with pytest.raises(dect.DectError, match="E_ARG"):
        dect._check(dect.lib().dect_project(plan.handle, dect._ptr(img), dect._ptr(img), 3,
                                            dect._stream()))
    pr = S.tiny_problem(0)
    p2 = dect.Plan(pr.geom, pr.spec, F32)
    meas = [dev(m, F32) for m in _meas(pr)]
    st = p2.new_state()
    with pytest.raises(dect.DectError, match="E_ARG"):
        p2.admm_init(meas, st, dect.AdmmParams(lm_iters=0))
    p2.admm_init(meas, st, dect.AdmmParams())
    with pytest.raises(dect.DectError, match="E_ARG"):
        p2.admm_iterate(meas, st, dect.AdmmParams(rho_mode=dect.RHO_SCHEDULE,
                                                  rho_schedule=[(1e-3, 1e-3)]), 3)
