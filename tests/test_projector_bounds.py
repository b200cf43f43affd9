"""The projector's index arithmetic checked on the host, for every workgroup, wave and
lane of a launch (tests/projector_bounds.cpp, built with g++ from the kernel's own
helpers in projidx.h): every sample of every ray lies on an image line, is taken by
exactly one wave, and every tap the kernel loads lies inside that line; the only exit
before the workgroup barrier is taken by whole workgroups.  Run on the geometries of
the GPU tests (including the FP64 parallel-beam 48^2 and 64^2 plans on which an earlier
four-samples-per-trip variant of the projector stalled) and of the benchmark."""
import math
import os
import shutil
import subprocess

import pytest

from paper_1905_00934_amd import synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sym(g):
    full = abs(g["span"] - 2 * math.pi) < 1e-12
    return 4 if (g["kind"] == "fan" and full and g["n_views"] % 4 == 0 and g["nx"] == g["ny"]
                 and g["nx"] % 2 == 0) else 1


CASES = {
    "starved_parallel48_f64": (S.geometry("parallel", 48, 48, 0.5, 60, 71, 0.5), 64),
    "tiny_parallel64_f64": (S.geometry("parallel", 64, 64, 0.5, 90, 95, 0.5), 64),
    "tiny_parallel64_f32": (S.geometry("parallel", 64, 64, 0.5, 90, 95, 0.5), 32),
    "sym_fan64_f64": (S.fan_geometry_fov(64, 120, 100, fov_cm=25.6, src_iso_cm=40.0,
                                         src_det_cm=70.0), 64),
    "ragged_fan_f64": (S.geometry("fan", 37, 29, 0.4, 50, 71, 0.45, det_offset=0.3,
                                  src_iso_cm=30.0, src_det_cm=52.0, angle0=0.1), 64),
    "ragged_parallel_f64": (S.geometry("parallel", 33, 47, 0.5, 41, 300, 0.17,
                                       det_offset=-0.25, angle0=0.05), 64),
    "sym_fan_offset_f64": (S.geometry("fan", 32, 32, 0.5, 44, 57, 0.6, det_offset=0.37,
                                      src_iso_cm=30.0, src_det_cm=50.0, angle0=0.2), 64),
    "one_view_parallel_f64": (S.geometry("parallel", 7, 5, 0.5, 1, 9, 0.5, angle0=0.3), 64),
    "two_by_two_f64": (S.geometry("parallel", 2, 2, 1.0, 7, 5, 0.8), 64),
    "fan256_f32": (S.fan_geometry_fov(256, 360, 512), 32),
    "fan384_f32": (S.fan_geometry_fov(384, 540, 768), 32),
    "fan512_f32": (S.fan_geometry_fov(512, 720, 1024), 32),
}


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("pb") / "projector_bounds")
    cmd = ["g++", "-std=c++17", "-O2", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1905_00934_amd", "csrc"),
           os.path.join(ROOT, "tests", "projector_bounds.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("name", list(CASES))
def test_projector_indices_stay_in_bounds(checker, name):
    g, prec = CASES[name]
    kind = 0 if g["kind"] == "parallel" else 1
    args = [str(v) for v in (kind, g["nx"], g["ny"], g["pixel_cm"], g["n_views"], g["n_det"],
                             g["det_cm"], g["det_offset"], g["src_iso_cm"], g["src_det_cm"],
                             g["angle0"], g["span"], _sym(g), prec)]
    r = subprocess.run([checker, *args], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("OK")
