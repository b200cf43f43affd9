"""The LM(m) x CG(n) baseline (Eqs. (7)-(8)) on the GPU against the oracle.

Tolerances: FP64 images to 1e-8 relative L2 with the same rho sequence and accept
decisions (the logged data terms to 1e-9); FP32 at 512x512 after 2 iterations with
fixed rho: x_c 1e-3, x_p 5e-3.
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = {"tiny": (None, 1, 1, 6), "sym_fan": (SYM_FAN, 2, 2, 4), "ragged": (RAGGED, 1, 3, 4)}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mode", ["adaptive", "fixed"])
def test_lmcg_fp64_matches_oracle(dect, name, mode):
    g, m, n, its = CASES[name]
    pr = S.tiny_problem(0) if g is None else _problem(g, 5)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    prm = O.Params(lm_iters=m, cg_iters=n, rho_mode=mode)
    ost = orc.lmcg_iterate(orc.lmcg_init(mh, ml, wh, wl, prm), mh, ml, wh, wl, prm, its)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    meas = [_dev(v, F64) for v in (mh, ml, wh, wl)]
    params = dect.AdmmParams(lm_iters=m, cg_iters=n,
                             rho_mode=dect.RHO_ADAPTIVE if mode == "adaptive" else dect.RHO_FIXED)
    st = plan.new_lmcg_state()
    plan.lmcg_init(meas, st, params)
    log = plan.lmcg_iterate(meas, st, params, its, log=True)
    x = st.x.cpu().numpy()
    for b in range(2):
        assert _rel(x[b], ost.x[b]) <= 1e-8
        assert _rel(st.Rx[b].cpu().numpy(), ost.Rx[b]) <= 1e-8
    assert [e["rho"] for e in log] == [tuple(e["rho"]) for e in ost.log]
    for e, o in zip(log, ost.log):
        assert e["data"] == pytest.approx(o["data"], rel=1e-9)
        assert e["tv"] == pytest.approx(o["tv"], rel=1e-8, abs=1e-14)
        assert e["r"] == pytest.approx(tuple(o["r"]), rel=1e-8)


def test_lmcg_from_cdm_fbp_image_fp64_matches_oracle(dect):
    pr = _problem(RAGGED, 7)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    x0 = orc.cdm_fbp_start(mh, ml, wh, wl, 20)
    prm = O.Params(lm_iters=1, cg_iters=2)
    ost = orc.lmcg_iterate(orc.lmcg_init(mh, ml, wh, wl, prm, x0=x0), mh, ml, wh, wl, prm, 4)
    plan = dect.Plan(pr.geom, pr.spec, F64)
    meas = [_dev(v, F64) for v in (mh, ml, wh, wl)]
    params = dect.AdmmParams(lm_iters=1, cg_iters=2)
    st = plan.new_lmcg_state()
    plan.lmcg_init(meas, st, params, x0=_dev(np.moveaxis(x0, 0, -1), F64))
    log = plan.lmcg_iterate(meas, st, params, 4, log=True)
    x = st.x.cpu().numpy()
    for b in range(2):
        assert _rel(x[b], ost.x[b]) <= 1e-8
    assert [e["rho"] for e in log] == [tuple(e["rho"]) for e in ost.log]


def test_lmcg_fp32_full_size(dect):
    pr = S.slice_problem(0, with_image=False)
    orc = O.Oracle(pr.geom, pr.spec)
    mh, ml, wh, wl = _meas(pr)
    prm = O.Params(rho_mode="fixed")
    ost = orc.lmcg_iterate(orc.lmcg_init(mh, ml, wh, wl, prm), mh, ml, wh, wl, prm, 2)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    meas = [_dev(v, F32) for v in (mh, ml, wh, wl)]
    params = dect.AdmmParams(rho_mode=dect.RHO_FIXED)
    st = plan.new_lmcg_state()
    plan.lmcg_init(meas, st, params)
    plan.lmcg_iterate(meas, st, params, 2)
    x = st.x.double().cpu().numpy()
    e = [_rel(x[b], ost.x[b]) for b in range(2)]
    assert e[0] <= 1e-3 and e[1] <= 5e-3, e


def test_lmcg_zero_image_equals_default_start(dect):
    pr = _problem(SYM_FAN, 2)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    meas = [_dev(v, F32) for v in _meas(pr)]
    params = dect.AdmmParams(cg_iters=2)
    s1, s2 = plan.new_lmcg_state(), plan.new_lmcg_state()
    plan.lmcg_init(meas, s1, params)
    plan.lmcg_init(meas, s2, params, x0=torch.zeros((plan.ny, plan.nx, 2), dtype=F32,
                                                     device="cuda"))
    plan.lmcg_iterate(meas, s1, params, 3)
    plan.lmcg_iterate(meas, s2, params, 3)
    torch.cuda.synchronize()
    for k in ("x", "y", "uy", "z", "uz", "Rx"):
        assert torch.equal(getattr(s1, k), getattr(s2, k)), k
    sc = slice(s1.layout.scalars, s1.layout.scalars + 24 * 8)
    assert torch.equal(s1.buf[sc], s2.buf[sc])


def test_lmcg_rejects_bad_params(dect):
    pr = S.tiny_problem(0)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    meas = [_dev(v, F32) for v in _meas(pr)]
    st = plan.new_lmcg_state()
    for bad in (dect.AdmmParams(precond=dect.PRECOND_RAMP),
                dect.AdmmParams(rho_mode=dect.RHO_SCHEDULE, rho_schedule=[(1e-3, 1e-3)] * 4),
                dect.AdmmParams(cg_iters=0)):
        with pytest.raises(dect.DectError):
            plan.lmcg_init(meas, st, bad)
