"""Failure handling on the GPU: non-finite inputs are reported, not hidden.

A NaN in the weights or the measurements makes the data cost of the a-update
(Eq. (13)) non-finite; the iteration log flags it and dect_admm_iterate returns
DECT_E_NONFINITE, and a served request whose counts hold a NaN ends with that
status at its first check while the other requests in flight finish normally.
No control flow of any kernel depends on the data (loop bounds and indices come
from the geometry and the tables), so such inputs cannot hang or fault a kernel.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_1905_00934_amd import synth as S

pytestmark = pytest.mark.gpu

F64, F32 = torch.float64, torch.float32
E_NONFINITE = -5


@pytest.fixture(scope="module")
def dect():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00934_amd import dect as D
    D.lib()
    return D


def _meas(pr):
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    return [mh, ml, wh, wl]


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("which", [0, 3])  # m_h or w_l
def test_admm_iterate_reports_nonfinite_input(dect, dtype, which):
    pr = S.tiny_problem(0)
    plan = dect.Plan(pr.geom, pr.spec, dtype)
    meas = _meas(pr)
    bad = [m.copy() for m in meas]
    bad[which][17, 40] = np.nan
    dm = [torch.from_numpy(m).to("cuda", dtype) for m in bad]
    params = dect.AdmmParams()
    st = plan.new_state()
    plan.admm_init(dm, st, params)
    with pytest.raises(dect.DectError) as e:
        plan.admm_iterate(dm, st, params, 2, log=True)
    assert e.value.status == E_NONFINITE
    log = plan.state_log(st, 0, 2)
    assert all(r["flags"] & 1 for r in log)
    assert not np.isfinite(log[-1]["data"])
    # The library keeps working: the same slice with clean inputs runs and logs finite
    # values on the same stream.
    good = [torch.from_numpy(m).to("cuda", dtype) for m in meas]
    st2 = plan.new_state()
    plan.admm_init(good, st2, params)
    log2 = plan.admm_iterate(good, st2, params, 2, log=True)
    assert all(r["flags"] == 0 and np.isfinite(r["data"]) for r in log2)


def test_server_reports_nonfinite_counts(dect):
    g = S.fan_geometry_fov(48, 88, 80, fov_cm=19.2, src_iso_cm=40.0, src_det_cm=70.0)
    ph = S.tiny_phantom(3)
    k = 48 * g["pixel_cm"] / 32.0
    ph = S.Phantom([S.Shape(sh.kind, k * sh.cx, k * sh.cy, k * sh.ax, k * sh.ay, sh.rot,
                            sh.xc, sh.xp) for sh in ph.shapes])
    pr = S.make_problem("sym_fan48", g, ph, 1e5, 3, with_image=False)
    plan = dect.Plan(g, pr.spec, F32)
    ch_bad = pr.counts_high.copy()
    ch_bad[5, 33] = np.nan
    srv = dect.Server(max_slots=4, step_iters=3)
    t_bad = srv.submit(plan, ch_bad, pr.counts_low, pr.i0, tol=0.0, max_iters=12)
    t_good = srv.submit(plan, pr.counts_high, pr.counts_low, pr.i0, tol=0.0, max_iters=12)
    (_, r_bad), (x_good, r_good) = srv.wait(t_bad, 60000), srv.wait(t_good, 60000)
    st = srv.stats()
    srv.close()
    assert r_bad["status"] == E_NONFINITE
    assert r_bad["iters"] == 3  # stopped at its first check
    assert r_good["status"] == 0 and r_good["iters"] == 12
    assert np.isfinite(x_good).all() and np.isfinite(r_good["objective"])
    assert st["completed"] == 2 and st["in_flight"] == 0
