"""Degenerate and boundary cases of the HIP path against the oracle.

Starved rays (zero counts behind metal, so w = 0 and m = ln I0), an empty phantom,
the smallest plans (2x2 images, one view, one detector bin), the preconditioner's
size limit and zero-iteration calls.  FP64 tolerances as in the parity tests:
operators 1e-12 of the largest value, ADMM images 1e-8 with the same rho sequence.
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


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def _meas(pr):
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    return mh, ml, wh, wl


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


SMALL = {
    "parallel_2x2": S.geometry("parallel", 2, 2, 1.0, 4, 3, 1.0),
    "fan_2x2_sym": S.geometry("fan", 2, 2, 1.0, 8, 5, 0.8, src_iso_cm=10.0, src_det_cm=18.0),
    "parallel_one_view": S.geometry("parallel", 7, 5, 0.5, 1, 9, 0.5, angle0=0.3),
    "fan_one_bin": S.geometry("fan", 6, 6, 0.5, 12, 1, 0.4, src_iso_cm=12.0, src_det_cm=20.0),
}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("ch", [1, 2])
def test_smallest_plans_project_backproject(dect, name, ch):
    g = SMALL[name]
    orc = O.Oracle(g, S.default_spectra())
    plan = dect.Plan(g, S.default_spectra(), F64)
    ny, nx = orc.img_shape
    V, D = orc.sino_shape
    rng = np.random.default_rng(3)
    img = rng.random((ny, nx, ch))
    sino = rng.random((V, D, ch))
    shape_i = (ny, nx) if ch == 1 else (ny, nx, ch)
    shape_s = (V, D) if ch == 1 else (V, D, ch)
    Rg = plan.project(_dev(img.reshape(shape_i), F64)).cpu().numpy().reshape(V, D, ch)
    Bg = plan.backproject(_dev(sino.reshape(shape_s), F64)).cpu().numpy().reshape(ny, nx, ch)
    for c in range(ch):
        want_r = orc.project(img[..., c], count=None)
        want_b = orc.backproject(sino[..., c], count="RT_dual")
        assert np.max(np.abs(Rg[..., c] - want_r)) <= 1e-12 * max(np.abs(want_r).max(), 1.0)
        assert np.max(np.abs(Bg[..., c] - want_b)) <= 1e-12 * max(np.abs(want_b).max(), 1.0)


def _admm_pair(dect, pr, n_iter, prm_kw=None, dtype=F64):
    prm_kw = prm_kw or {}
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    prm = O.Params(**prm_kw)
    ost = orc.admm_iterate(orc.admm_init(mh, ml, wh, wl, prm), mh, ml, wh, wl, prm, n_iter)
    plan = dect.Plan(pr.geom, pr.spec, dtype)
    meas = [_dev(v, dtype) for v in (mh, ml, wh, wl)]
    params = dect.AdmmParams(**prm_kw)
    st = plan.new_state()
    plan.admm_init(meas, st, params)
    log = plan.admm_iterate(meas, st, params, n_iter, log=True)
    return ost, st, log


def test_starved_rays_fp64_admm_matches_oracle(dect):
    """A steel disk at low dose: some rays count zero photons in both spectra."""
    g = S.geometry("parallel", 48, 48, 0.5, 60, 71, 0.5)
    ph = S.Phantom([S.Shape("ellipse", 0.0, 0.0, 9.0, 7.0, 0.2, 0.2, 0.02),
                    S.Shape("ellipse", 2.0, -1.0, 2.5, 2.5, 0.0, 2.0, 5.0)])
    pr = S.make_problem("starved", g, ph, 300.0, 11, with_image=False)
    mh, ml, wh, wl = _meas(pr)
    starved = (wh == 0) & (wl == 0)
    assert starved.sum() >= 20, "the case needs rays with no photons in either spectrum"
    ost, st, log = _admm_pair(dect, pr, 5, dict(cg_iters=2, lm_iters=2))
    x = st.x.cpu().numpy()
    for b in range(2):
        assert _rel(x[..., b], ost.x[b]) <= 1e-8
    assert [e["rho"] for e in log] == [tuple(e["rho"]) for e in ost.log]
    assert all(e["flags"] == 0 for e in log)


def test_starved_rays_decomposition_fp64(dect):
    """With w = 0 the decomposition is the proximal step alone: a tends to v."""
    g = S.geometry("parallel", 16, 16, 0.5, 8, 21, 0.5)
    orc = O.Oracle(g, S.default_spectra())
    plan = dect.Plan(g, S.default_spectra(), F64)
    V, D = orc.sino_shape
    rng = np.random.default_rng(2)
    mh, ml = rng.random((V, D)) * 3, rng.random((V, D)) * 3
    wh, wl = np.zeros((V, D)), np.zeros((V, D))
    vc, vp = rng.random((V, D)), rng.random((V, D)) * 0.1
    a0 = np.stack(orc.linearised(mh, ml), -1)
    a = _dev(a0, F64)
    plan.decompose_rays(*(_dev(m, F64) for m in (mh, ml, wh, wl)), a,
                        _dev(np.stack([vc, vp], -1), F64), (1e-3, 2e-3), 3)
    wc, wp, _ = orc.udm(mh, ml, wh, wl, vc, vp, 1e-3, 2e-3, 3, a0[..., 0], a0[..., 1])
    got = a.cpu().numpy()
    np.testing.assert_allclose(got[..., 0], wc, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(got[..., 1], wp, rtol=1e-12, atol=1e-12)
    # Each accepted damped step leaves mu/(1+mu) of the distance to v (mu = 1e-3, 1e-4,
    # 1e-5), so after three iterations |a - v| is ~1e-12 of the start's distance.
    for c, v in ((0, vc), (1, vp)):
        assert np.all(np.abs(got[..., c] - v) <= 2e-12 * np.abs(a0[..., c] - v) + 1e-15)


def test_empty_phantom_fp64_admm_matches_oracle(dect):
    g = S.geometry("fan", 32, 32, 0.5, 40, 61, 0.5, src_iso_cm=30.0, src_det_cm=50.0)
    pr = S.make_problem("empty", g, S.Phantom([]), 1e5, 4, with_image=False)
    ost, st, log = _admm_pair(dect, pr, 4, dict(cg_iters=2))
    x = st.x.cpu().numpy()
    for b in range(2):
        # Only noise is reconstructed: compare absolutely, on the oracle's scale.
        assert np.max(np.abs(x[..., b] - ost.x[b])) <= 1e-8 * max(np.abs(ost.x[b]).max(), 1e-6)
    assert [e["rho"] for e in log] == [tuple(e["rho"]) for e in ost.log]


def test_zero_iterations_leave_the_state_unchanged(dect):
    pr = S.tiny_problem(1)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    meas = [_dev(v, F32) for v in _meas(pr)]
    params = dect.AdmmParams()
    st = plan.new_state()
    plan.admm_init(meas, st, params)
    torch.cuda.synchronize()
    before = st.buf.clone()
    assert plan.admm_iterate(meas, st, params, 0, log=True) == []
    torch.cuda.synchronize()
    assert torch.equal(before, st.buf)
    lst = plan.new_lmcg_state()
    plan.lmcg_init(meas, lst, params)
    torch.cuda.synchronize()
    x0 = lst.x.clone()
    plan.lmcg_iterate(meas, lst, params, 0)
    torch.cuda.synchronize()
    assert torch.equal(x0, lst.x)


def test_preconditioner_size_limit(dect):
    """Images whose padded side exceeds the FFT limit have no preconditioner."""
    g = S.geometry("parallel", 1100, 8, 0.1, 4, 16, 0.1)
    plan = dect.Plan(g, S.default_spectra(), F32)
    with pytest.raises(dect.DectError) as e:
        plan.precondition(torch.zeros((8, 1100, 2), dtype=F32, device="cuda"))
    assert "DECT_E_SHAPE" in str(e.value)
    V, D = 4, 16
    meas = [torch.zeros((V, D), dtype=F32, device="cuda") for _ in range(4)]
    st = plan.new_state()
    with pytest.raises(dect.DectError):
        plan.admm_init(meas, st, dect.AdmmParams(precond=dect.PRECOND_RAMP))
        plan.admm_iterate(meas, st, dect.AdmmParams(precond=dect.PRECOND_RAMP), 1)
