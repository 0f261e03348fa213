"""The host part of plan creation (system checks, screening, canonical pairs,
task lists, workspace chunks, mixed-precision lists) compiled on its own with
AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only) and run
on clusters, a batch and periodic cells, with and without a workspace budget;
its pair, chunk and workspace counts equal the library's host-only plans."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2403_10343_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "plan_sanitize")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(ROOT, "tests", "plan_sanitize_main.cpp"),
           os.path.join(CSRC, "exx_plan.cpp"), os.path.join(CSRC, "exx_plan_periodic.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def _write(path, sysm, budget):
    n, nsys = sysm.n_atoms, sysm.n_systems
    with open(path, "wb") as f:
        f.write(struct.pack("=4i", n, len(sysm.basis_table), nsys, 1 if sysm.lattice is not None else 0))
        f.write(struct.pack("=dq", float(sysm.r_cut), int(budget)))
        f.write(np.ascontiguousarray(sysm.species, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(sysm.pos, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(sysm.basis_table, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(sysm.aux_table, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(sysm.sys_off, dtype=np.int32).tobytes())
        if sysm.lattice is not None:
            f.write(np.ascontiguousarray(sysm.lattice, dtype=np.float64).tobytes())


def _tiny():
    lat = np.array([[3.0, 0.0, 0.0], [0.4, 3.2, 0.0], [0.2, -0.3, 3.4]])
    pos = np.array([[0.2, 0.3, 0.1], [2.6, 0.5, 0.4], [1.3, 2.9, 3.0], [1.5, 1.6, 1.7], [0.5, 2.8, 3.2]])
    return synth.System(np.array([0, 1, 1, 0, 1]), pos, 1.45, 3, lattice=lat)


CASES = {
    "cluster": (lambda: synth.water_cluster(8, 5), 0),
    "ice192_chunked": (lambda: synth.ice_box(2, 2, 2, seed=3), 3),
    "batch": (lambda: synth.cluster_batch(4, n_min=6, n_max=30), 0),
    "tiny_periodic": (_tiny, 0),
    "ice_cell_chunked": (lambda: synth.ice_box_periodic(1, 1, 1, seed=4, r_cut=3.4), 2),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_host_plan_code_under_sanitizers(driver, tmp_path, name):
    from paper_2403_10343_amd import Plan
    make, frac = CASES[name]
    sysm = make()
    full = Plan.for_system(sysm, host_only=True)
    budget = full.info["intermediate_bytes_stored"] // frac if frac else 0
    plan = Plan.for_system(sysm, host_only=True, ws_budget_bytes=budget)
    path = str(tmp_path / "system.bin")
    _write(path, sysm, budget)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, path], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    n_pairs, n_chunks, inter = (int(x) for x in r.stdout.split())
    assert n_pairs == plan.info["n_pairs"]
    assert n_chunks == plan.info["n_chunks"] and inter == plan.info["intermediate_bytes"]
    if frac:
        assert n_chunks >= 2
