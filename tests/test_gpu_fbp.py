"""The CDM-FBP baseline and the ADMM start from its image, HIP against the oracle.

Tolerances: FP64 CDM line integrals to 1e-9 relative L2 (both sides run the same
active-set LM in double precision); FP64 FBP to 1e-11 of the image's largest value;
FP32 at full size: FBP to 1e-5 relative L2, CDM to 1e-4 (c) and 1e-3 (p) with
rays that took another accept/reject branch under 0.1 %; FP64 ADMM started from
the CDM-FBP image to 1e-8 with the same rho sequence.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_1905_00934_amd import synth as S

pytestmark = pytest.mark.gpu

F64, F32 = torch.float64, torch.float32

SYM_FAN = S.fan_geometry_fov(64, 120, 100, fov_cm=25.6, src_iso_cm=40.0, src_det_cm=70.0)
RAGGED = S.geometry("fan", 37, 29, 0.4, 50, 71, 0.45, det_offset=0.3, src_iso_cm=30.0,
                    src_det_cm=52.0, angle0=0.1)
PARALLEL = S.geometry("parallel", 48, 40, 0.5, 60, 97, 0.5, det_offset=-0.2, angle0=0.05)


@pytest.fixture(scope="module")
def dect():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00934_amd import dect as D
    D.lib()
    return D


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def _meas(pr):
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    return mh, ml, wh, wl


def _problem(g, seed):
    k = min(g["nx"], g["ny"]) * g["pixel_cm"] / 32.0
    ph = S.tiny_phantom(seed)
    ph = S.Phantom([S.Shape(sh.kind, k * sh.cx, k * sh.cy, k * sh.ax, k * sh.ay, sh.rot,
                            sh.xc, sh.xp) for sh in ph.shapes])
    return S.make_problem("p", g, ph, 1e5, seed, with_image=False)


def _case(name):
    if name == "tiny":
        return S.tiny_problem(0)
    return _problem({"sym_fan": SYM_FAN, "ragged": RAGGED, "parallel": PARALLEL}[name], 3)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["tiny", "sym_fan", "ragged", "parallel"])
def test_cdm_fp64_matches_oracle(dect, name):
    pr = _case(name)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    wc, wp = orc.cdm(mh, ml, wh, wl, 20)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    cost = torch.empty(mh.shape, dtype=F64, device="cuda")
    a = plan.cdm(*(_dev(m, F64) for m in (mh, ml, wh, wl)), lm_iters=20, cost=cost)
    got = a.cpu().numpy()
    assert got.min() >= 0.0
    assert _rel(got[..., 0], wc) <= 1e-9
    assert _rel(got[..., 1], wp) <= 1e-9
    want_cost = orc.data_cost(wc, wp, mh, ml, wh, wl)
    assert float(cost.sum()) == pytest.approx(want_cost, rel=1e-9)


def test_cdm_zero_iterations_is_projected_linearisation(dect):
    pr = _case("ragged")
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    c0, p0 = orc.linearised(mh, ml)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    got = plan.cdm(*(_dev(m, F64) for m in (mh, ml, wh, wl)), lm_iters=0).cpu().numpy()
    np.testing.assert_allclose(got[..., 0], np.maximum(c0, 0.0), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(got[..., 1], np.maximum(p0, 0.0), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("name", ["sym_fan", "ragged", "parallel"])
@pytest.mark.parametrize("ch", [1, 2])
def test_fbp_fp64_matches_oracle(dect, name, ch):
    g = {"sym_fan": SYM_FAN, "ragged": RAGGED, "parallel": PARALLEL}[name]
    orc = O.Oracle(g, S.default_spectra())
    V, D = orc.sino_shape
    rng = np.random.default_rng(11 + ch)
    sino = rng.random((V, D, ch)) if ch == 2 else rng.random((V, D))
    plan = dect.Plan(g, S.default_spectra(), F64)
    got = plan.fbp(_dev(sino, F64)).cpu().numpy()
    if ch == 1:
        want = orc.fbp(sino)
    else:
        want = np.stack([orc.fbp(sino[..., 0]), orc.fbp(sino[..., 1])], -1)
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


def test_fbp_fp32_full_size(dect):
    pr = S.slice_problem(0, with_image=False)
    orc = O.Oracle(pr.geom, pr.spec)
    ac, ap = pr.a_true
    want = orc.fbp(ac)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    got = plan.fbp(_dev(ac, F32)).double().cpu().numpy()
    assert _rel(got, want) <= 1e-5


def test_cdm_fp32_full_size_sampled(dect):
    pr = S.slice_problem(0, with_image=False)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    got = plan.cdm(*(_dev(m, F32) for m in (mh, ml, wh, wl)), lm_iters=20).double().cpu().numpy()
    # Every 13th ray: the oracle decomposes rays independently.
    sel = np.arange(0, mh.size, 13)
    wc, wp = orc.cdm(*(m.ravel()[sel] for m in (mh, ml, wh, wl)), 20)
    gc, gp = got[..., 0].ravel()[sel], got[..., 1].ravel()[sel]
    assert got.min() >= 0.0
    assert _rel(gc, wc) <= 1e-4 and _rel(gp, wp) <= 1e-3
    far = np.abs(gc - wc) > 1e-3 * (np.abs(wc) + 1)
    assert far.mean() < 1e-3


@pytest.mark.parametrize("name", ["tiny", "ragged"])
def test_cdm_fbp_start_fp64_matches_oracle(dect, name):
    pr = _case(name)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    (wc, wp), wimg = orc.cdm_fbp(mh, ml, wh, wl, 20)
    wx0 = orc.cdm_fbp_start(mh, ml, wh, wl, 20)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    a, img, x0 = plan.cdm_fbp_start([_dev(m, F64) for m in (mh, ml, wh, wl)], 20)
    a, img, x0 = a.cpu().numpy(), img.cpu().numpy(), x0.cpu().numpy()
    assert _rel(a[..., 0], wc) <= 1e-9 and _rel(a[..., 1], wp) <= 1e-9
    for b in range(2):
        assert np.max(np.abs(img[..., b] - wimg[b])) <= 1e-9 * np.max(np.abs(wimg[b]))
        assert np.max(np.abs(x0[..., b] - wx0[b])) <= 1e-9 * np.max(np.abs(wx0[b]))


@pytest.mark.parametrize("name", ["tiny", "sym_fan", "ragged"])
def test_admm_from_cdm_fbp_image_fp64_matches_oracle(dect, name):
    pr = _case(name)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    x0 = orc.cdm_fbp_start(mh, ml, wh, wl, 20)
    prm = O.Params(cg_iters=2, lm_iters=2)
    ost = orc.admm_iterate(orc.admm_init(mh, ml, wh, wl, prm, x0=x0), mh, ml, wh, wl, prm, 5)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    meas = [_dev(m, F64) for m in (mh, ml, wh, wl)]
    params = dect.AdmmParams(cg_iters=2, lm_iters=2)
    st = plan.new_state()
    plan.admm_init(meas, st, params, x0=_dev(np.moveaxis(x0, 0, -1), F64))
    log = plan.admm_iterate(meas, st, params, 5, log=True)
    x = st.x.cpu().numpy()
    for b in range(2):
        assert _rel(x[..., b], ost.x[b]) <= 1e-8
    assert [e["rho"] for e in log] == [tuple(e["rho"]) for e in ost.log]


def test_admm_from_zero_image_equals_plain_init(dect):
    pr = _case("sym_fan")
    plan = dect.Plan(pr.geom, pr.spec, F32)
    meas = [_dev(m, F32) for m in _meas(pr)]
    params = dect.AdmmParams(cg_iters=2)
    s1, s2 = plan.new_state(), plan.new_state()
    plan.admm_init(meas, s1, params)
    plan.admm_init(meas, s2, params, x0=torch.zeros((plan.ny, plan.nx, 2), dtype=F32,
                                                     device="cuda"))
    plan.admm_iterate(meas, s1, params, 3)
    plan.admm_iterate(meas, s2, params, 3)
    torch.cuda.synchronize()
    assert torch.equal(s1.x, s2.x) and torch.equal(s1.a, s2.a)


def test_fbp_errors(dect):
    plan = dect.Plan(SYM_FAN, S.default_spectra(), F32)
    sino = torch.zeros((plan.V, plan.D, 3), dtype=F32, device="cuda")
    img = torch.zeros((plan.ny, plan.nx, 3), dtype=F32, device="cuda")
    st = dect.lib().dect_fbp(plan.handle, dect._ptr(sino), dect._ptr(img), 3, None)
    assert dect.STATUS[st] == "DECT_E_ARG"
    # A row padded to more than 4096 entries has no filter.
    wide = S.geometry("parallel", 8, 8, 1.0, 4, 2100, 0.01)
    wplan = dect.Plan(wide, S.default_spectra(), F32)
    with pytest.raises(dect.DectError):
        wplan.fbp(torch.zeros((4, 2100), dtype=F32, device="cuda"))
