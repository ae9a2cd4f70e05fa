"""Host code under the address and undefined-behaviour sanitizers (CPU only).

- The tiled-layout construction the library runs once per mesh (node
  numbering, tet order, tiles, the dealing of tets to lanes, node -> entry
  lists; paper_2103_16747_amd/csrc/layout.h) is compiled with g++
  -fsanitize=address,undefined into tests/layout_check.cpp's checker and run
  on the block and fingertip meshes at several tile limits; the checker also
  asserts the layout's invariants and reports how well the dealing spreads
  each 16-lane group's LDS accesses over the banks.
- The FP64 oracle (oracle/oracle.c) is compiled with the same sanitizers and
  its pin tests run against that build in a child process with the sanitizer
  runtime preloaded.
Any sanitizer report aborts the child and fails the test.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2103_16747_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip(f"{name} not available")
    return p


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


@pytest.fixture(scope="module")
def layout_checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "layout_check")
    subprocess.run(["g++", "-std=c++17", "-pthread", *SAN, "-o", exe, os.path.join(ROOT, "tests", "layout_check.cpp")],
                   check=True)
    return exe


def _write_mesh(path, mesh):
    with open(path, "wb") as f:
        np.array([mesh.n, mesh.m], dtype=np.int32).tofile(f)
        np.ascontiguousarray(mesh.X, dtype=np.float64).tofile(f)
        np.ascontiguousarray(mesh.tets, dtype=np.int32).tofile(f)


MESHES = {
    "cube8": W.cube_block_mesh,
    "fingertip5k": lambda: W.fingertip_mesh(5000),
    "fingertip20k": lambda: W.fingertip_mesh(20000),
    "graded_block": lambda: W.block_mesh(xs=np.geomspace(1e-4, 1e-2, 7), ys=np.linspace(0, 4e-3, 5),
                                         zs=np.linspace(0, 2e-3, 4)),
}


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("limits", [(512, 256), (256, 128), (64, 16)])
def test_layout_construction_under_sanitizers(layout_checker, tmp_path, name, limits):
    mesh = MESHES[name]()
    path = str(tmp_path / f"{name}.bin")
    _write_mesh(path, mesh)
    p = subprocess.run([layout_checker, path, str(limits[0]), str(limits[1])], capture_output=True, text=True,
                       env=_env(), timeout=300)
    assert p.returncode == 0 and p.stdout.startswith("ok"), (p.stdout, p.stderr[-2000:])
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr
    if name.startswith("fingertip") and limits[1] >= 128:
        # the dealing leaves (almost) no repeated LDS bank in a 16-lane group
        passes = float(p.stdout.split("passes=")[1].split()[0])
        assert passes <= 1.05, p.stdout


def test_oracle_pins_under_sanitizers():
    import oracle

    oracle.build(force=True, sanitize=True)
    env = _env()
    env["ORACLE_SANITIZED"] = "1"
    env["LD_PRELOAD"] = ":".join([_runtime("libasan.so"), _runtime("libubsan.so")])
    # the pins, minus the three refinement studies (minutes under the sanitizers)
    tests = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_pins.py", "test_oracle_corotational.py", "test_oracle_friction.py",
              "test_oracle_dynamics.py", "test_oracle_outputs.py")]
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "-k", "not hertz and not flat_punch", *tests],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    assert p.returncode == 0, (p.stdout[-3000:], p.stderr[-3000:])
    assert "runtime error" not in p.stdout + p.stderr
