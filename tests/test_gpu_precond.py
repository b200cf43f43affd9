"""The ramp preconditioner (2-D FFT in HIP) and preconditioned CG against the oracle.

Tolerances: FP64 preconditioner to 1e-12 of the largest value; FP32 at 512x512
to 1e-5 relative L2; FP64 ADMM with PCG to 1e-8 with the same rho sequence; FP32
512x512 after 3 iterations with the oracle's rho sequence: x_c 1e-3, x_p 5e-3.
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


def _oracle_precond(img2):
    f = O.ramp_filter(*O.pad_shape(*img2.shape[:2]))
    return np.stack([O.precondition(img2[..., 0], f), O.precondition(img2[..., 1], f)], -1)


@pytest.mark.parametrize("ny,nx", [(29, 37), (64, 64), (60, 100), (2, 2), (7, 5)])
def test_precondition_fp64_matches_oracle(dect, ny, nx):
    g = S.geometry("parallel", nx, ny, 0.5, 12, max(nx, ny) * 2, 0.5)
    plan = dect.Plan(g, S.default_spectra(), F64)
    img = np.random.default_rng(ny * 1000 + nx).standard_normal((ny, nx, 2))
    got = plan.precondition(_dev(img, F64)).cpu().numpy()
    want = _oracle_precond(img)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_precondition_fp32_full_size(dect):
    g = S.fan_geometry_fov(512, 720, 1024)
    plan = dect.Plan(g, S.default_spectra(), F32)
    img = np.random.default_rng(5).standard_normal((512, 512, 2))
    got = plan.precondition(_dev(img, F32)).double().cpu().numpy()
    want = _oracle_precond(img)
    for c in range(2):
        err = np.linalg.norm(got[..., c] - want[..., c]) / np.linalg.norm(want[..., c])
        assert err <= 1e-5, err


def _meas(pr):
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    return mh, ml, wh, wl


def _shrunk_problem(g, seed):
    k = min(g["nx"], g["ny"]) * g["pixel_cm"] / 32.0
    ph = S.tiny_phantom(seed)
    ph = S.Phantom([S.Shape(sh.kind, k * sh.cx, k * sh.cy, k * sh.ax, k * sh.ay, sh.rot,
                            sh.xc, sh.xp) for sh in ph.shapes])
    return S.make_problem("p", g, ph, 1e5, seed, with_image=False)


@pytest.mark.parametrize("case", ["tiny", "sym_fan", "ragged"])
def test_admm_pcg_fp64_matches_oracle(dect, case):
    if case == "tiny":
        pr, n_it, cg, lm = S.tiny_problem(0), 10, 1, 1
    elif case == "sym_fan":
        g = S.fan_geometry_fov(64, 120, 100, fov_cm=25.6, src_iso_cm=40.0, src_det_cm=70.0)
        pr, n_it, cg, lm = _shrunk_problem(g, 4), 6, 3, 2
    else:
        g = S.geometry("fan", 37, 29, 0.4, 50, 71, 0.45, det_offset=0.3, src_iso_cm=30.0,
                       src_det_cm=52.0, angle0=0.1)
        pr, n_it, cg, lm = _shrunk_problem(g, 6), 6, 2, 1
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    prm = O.Params(cg_iters=cg, lm_iters=lm, precond="ramp")
    ost = orc.admm_iterate(orc.admm_init(mh, ml, wh, wl, prm), mh, ml, wh, wl, prm, n_it)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    meas = [_dev(m, F64) for m in (mh, ml, wh, wl)]
    params = dect.AdmmParams(cg_iters=cg, lm_iters=lm, precond=dect.PRECOND_RAMP)
    st = plan.new_state()
    plan.admm_init(meas, st, params)
    log = plan.admm_iterate(meas, st, params, n_it, log=True)
    x = st.x.cpu().numpy()
    for b in range(2):
        err = np.linalg.norm(x[..., b] - ost.x[b]) / np.linalg.norm(ost.x[b])
        assert err <= 1e-8, err
    assert [e["rho"] for e in log] == [tuple(e["rho"]) for e in ost.log]


def test_admm_pcg_fp32_full_size(dect):
    pr = S.slice_problem(0, with_image=False)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    prm = O.Params(precond="ramp")
    ost = orc.admm_iterate(orc.admm_init(mh, ml, wh, wl, prm), mh, ml, wh, wl, prm, 3)
    sched = [tuple(e["rho"]) for e in ost.log] + [tuple(ost.rho)]
    plan = dect.Plan(pr.geom, pr.spec, F32)
    meas = [_dev(m, F32) for m in (mh, ml, wh, wl)]
    params = dect.AdmmParams(rho_mode=dect.RHO_SCHEDULE, rho_schedule=sched,
                             precond=dect.PRECOND_RAMP)
    st = plan.new_state()
    plan.admm_init(meas, st, params)
    plan.admm_iterate(meas, st, params, 3)
    x = st.x.double().cpu().numpy()
    e = [np.linalg.norm(x[..., b] - ost.x[b]) / np.linalg.norm(ost.x[b]) for b in range(2)]
    assert e[0] <= 1e-3 and e[1] <= 5e-3, e


def test_batch_with_pcg_equals_alone(dect):
    g64 = S.fan_geometry_fov(64, 120, 100, fov_cm=25.6, src_iso_cm=40.0, src_det_cm=70.0)
    g48 = S.fan_geometry_fov(48, 88, 80, fov_cm=19.2, src_iso_cm=40.0, src_det_cm=70.0)
    pcg = dect.AdmmParams(cg_iters=2, precond=dect.PRECOND_RAMP)
    slices = []
    for g, seed in ((g64, 1), (g48, 2), (g64, 3)):
        pr = _shrunk_problem(g, seed)
        plan = dect.Plan(pr.geom, pr.spec, F32)
        meas = [_dev(m, F32) for m in _meas(pr)]
        s1, s2 = plan.new_state(), plan.new_state()
        plan.admm_init(meas, s1, pcg)
        plan.admm_init(meas, s2, pcg)
        slices.append((plan, meas, s1, s2))
    b = dect.Batch([(p, m, s2) for p, m, _, s2 in slices], pcg, graph=True)
    b.iterate(5)
    for p, m, s1, _ in slices:
        p.admm_iterate(m, s1, pcg, 5)
    torch.cuda.synchronize()
    for _, _, s1, s2 in slices:
        assert torch.equal(s1.buf, s2.buf)
    b.close()


def test_bad_precond_is_rejected(dect):
    pr = S.tiny_problem(0)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    meas = [_dev(m, F32) for m in _meas(pr)]
    st = plan.new_state()
    with pytest.raises(dect.DectError):
        plan.admm_init(meas, st, dect.AdmmParams(precond=7))
