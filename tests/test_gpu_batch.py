"""Batched slices (one launch per kernel per shape group, HIP-graph replay).

A slice's arithmetic and reduction order do not depend on the other slices of
its batch, so every slice's whole state after k batched iterations must be
bitwise equal to the state reached by k single-slice iterations on it alone.
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


def _meas(pr, dtype):
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    return [_dev(m, dtype) for m in (mh, ml, wh, wl)]


SMALL = {
    "sym_fan64": S.fan_geometry_fov(64, 120, 100, fov_cm=25.6, src_iso_cm=40.0, src_det_cm=70.0),
    "sym_fan48": S.fan_geometry_fov(48, 88, 80, fov_cm=19.2, src_iso_cm=40.0, src_det_cm=70.0),
    "ragged_fan": S.geometry("fan", 37, 29, 0.4, 50, 71, 0.45, det_offset=0.3,
                             src_iso_cm=30.0, src_det_cm=52.0, angle0=0.1),
}
# (geometry, seed): repeated geometries share one plan and one launch group.
MIX = [("sym_fan64", 0), ("sym_fan48", 1), ("sym_fan64", 2), ("ragged_fan", 3), ("sym_fan64", 4)]


def _problem(gname, seed):
    """The three-ellipse phantom (laid out for a 32 cm field) shrunk to this image."""
    g = SMALL[gname]
    k = min(g["nx"], g["ny"]) * g["pixel_cm"] / 32.0
    ph = S.tiny_phantom(seed)
    ph = S.Phantom([S.Shape(sh.kind, k * sh.cx, k * sh.cy, k * sh.ax, k * sh.ay, sh.rot,
                            sh.xc, sh.xp) for sh in ph.shapes])
    return S.make_problem(gname, g, ph, 1e5, seed, with_image=False)


def _setup(dect, dtype, params, mix):
    plans = {}
    out = []
    for gname, seed in mix:
        pr = _problem(gname, seed)
        if gname not in plans:
            plans[gname] = dect.Plan(pr.geom, pr.spec, dtype)
        plan = plans[gname]
        meas = _meas(pr, dtype)
        alone, batched = plan.new_state(), plan.new_state()
        plan.admm_init(meas, alone, params)
        plan.admm_init(meas, batched, params)
        out.append((plan, meas, alone, batched))
    return out


# Same image, ray count and grid sizes but different views and bins: the two plans
# fall into one launch group, whose kernels must take each slice's own sizes.
# 124 x 96 and 128 x 93 rays: 11904 each, 31 and 32 base views, projector grids of
# 3 x 16 workgroups at 2 base views per wave (4 x 8 at 4).
SMALL["sym_fan64_v124"] = S.fan_geometry_fov(64, 124, 96, fov_cm=25.6, src_iso_cm=40.0,
                                             src_det_cm=70.0)
SMALL["sym_fan64_v128"] = S.fan_geometry_fov(64, 128, 93, fov_cm=25.6, src_iso_cm=40.0,
                                             src_det_cm=70.0)


@pytest.mark.parametrize("dtype,rt_sums", [(F32, 0), (F64, 0), (F32, 1)])
def test_batch_group_of_different_view_and_bin_counts(dect, dtype, rt_sums):
    """(rt_sums 1: the FP32 transposes summing in double.)"""
    params = dect.AdmmParams(cg_iters=2, rt_sums=rt_sums)
    mix = [("sym_fan64_v124", 5), ("sym_fan64_v128", 6), ("sym_fan64_v124", 7)]
    sl = _setup(dect, dtype, params, mix)
    b = dect.Batch([(p, m, bs) for p, m, _, bs in sl], params, graph=True)
    assert b.groups == 1
    b.iterate(3)
    for p, m, alone, _ in sl:
        p.admm_iterate(m, alone, params, 3)
    torch.cuda.synchronize()
    for k, (p, m, alone, batched) in enumerate(sl):
        assert torch.equal(alone.buf, batched.buf), f"slice {k} ({mix[k][0]}) differs"
    b.close()


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_slices_equal_alone(dect, dtype, graph):
    params = dect.AdmmParams(rho0=(5e-3, 2e-2), cg_iters=2, lm_iters=2)
    sl = _setup(dect, dtype, params, MIX)
    b = dect.Batch([(p, m, bs) for p, m, _, bs in sl], params, graph=graph)
    assert b.groups == 3
    # Several calls with synchronisation and unrelated device work between the
    # replays; every replay must continue exactly where the previous one stopped.
    for n in (2, 1, 3):
        b.iterate(n)
        torch.cuda.synchronize()
        _ = (torch.ones(1000, device="cuda") * 3).sum().item()
    for p, m, alone, _ in sl:
        p.admm_iterate(m, alone, params, 6)
    torch.cuda.synchronize()
    for k, (p, m, alone, batched) in enumerate(sl):
        assert torch.equal(alone.buf, batched.buf), f"slice {k} ({MIX[k][0]}) differs"
    # The per-slice log is readable from the state.
    p, _, _, batched = sl[0]
    log = p.state_log(batched, 0, 6)
    assert [e["iter"] for e in log] == list(range(6))
    assert all(e["flags"] == 0 for e in log)
    with pytest.raises(dect.DectError):
        p.state_log(batched, 3, 4)   # iteration 6 has not run
    b.close()


def test_batch_full_size_graph_equals_alone(dect):
    """Two 512x512 slices and one 256x256 slice at the benchmark's launch shapes."""
    params = dect.AdmmParams()
    mix = [("slice512", 0), ("uneven", 0), ("slice512", 1)]
    plans, sl = {}, []
    for name, seed in mix:
        pr = (S.slice_problem(seed, with_image=False) if name == "slice512"
              else S.uneven_problem(seed, with_image=False))
        if name not in plans:
            plans[name] = dect.Plan(pr.geom, pr.spec, F32)
        plan = plans[name]
        meas = _meas(pr, F32)
        a, bst = plan.new_state(), plan.new_state()
        plan.admm_init(meas, a, params)
        plan.admm_init(meas, bst, params)
        sl.append((plan, meas, a, bst))
    b = dect.Batch([(p, m, bs) for p, m, _, bs in sl], params, graph=True)
    assert b.groups == 2
    b.iterate(3)
    for p, m, a, _ in sl:
        p.admm_iterate(m, a, params, 3)
    torch.cuda.synchronize()
    for k, (_, _, a, bst) in enumerate(sl):
        assert torch.equal(a.buf, bst.buf), f"slice {k} differs"
    b.close()


def test_pending_dual_rescale_settles_at_call_ends(dect):
    """The iterations leave the dual rescale after a change of rho pending for the readers
    of the duals and each call applies what is still pending: 20 calls of one iteration
    must give the state of one call of 20, bit for bit, with rho changing on the way."""
    params = dect.AdmmParams()
    pr = S.uneven_problem(0, with_image=False)
    plan = dect.Plan(pr.geom, pr.spec, F32)
    meas = _meas(pr, F32)
    one, many = plan.new_state(), plan.new_state()
    plan.admm_init(meas, one, params)
    plan.admm_init(meas, many, params)
    log = plan.admm_iterate(meas, one, params, 20, log=True)
    for _ in range(20):
        plan.admm_iterate(meas, many, params, 1)
    torch.cuda.synchronize()
    rhos = [e["rho"] for e in log]
    assert any(r != rhos[0] for r in rhos), "rho never changed: the test would be vacuous"
    assert torch.equal(one.buf, many.buf)
    assert one.scalars[2].item() == 1.0 and one.scalars[3].item() == 1.0  # nothing pending


def test_batch_argument_errors(dect):
    params = dect.AdmmParams()
    sl = _setup(dect, F32, params, MIX[:2])
    with pytest.raises(dect.DectError):   # a state used twice
        dect.Batch([(sl[0][0], sl[0][1], sl[0][3]), (sl[0][0], sl[0][1], sl[0][3])], params)
    sched = dect.AdmmParams(rho_mode=dect.RHO_SCHEDULE, rho_schedule=[(1e-3, 1e-3)] * 4)
    with pytest.raises(dect.DectError):   # schedules are single-slice only
        dect.Batch([(p, m, bs) for p, m, _, bs in sl], sched)
    with pytest.raises(dect.DectError):   # mixed precision
        p64 = dect.Plan(SMALL["sym_fan48"], S.default_spectra(), F64)
        st64 = p64.new_state()
        m64 = _meas(_problem("sym_fan48", 1), F64)
        dect.Batch([(sl[0][0], sl[0][1], sl[0][3]), (p64, m64, st64)], params)
