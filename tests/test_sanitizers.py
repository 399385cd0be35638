"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

Two drivers, compiled with g++ -fsanitize=address,undefined and
-fno-sanitize-recover=all so that any report fails the run:
  * tests/sanitize/oracle_main.cpp -- the oracle (oracle/lbrs_oracle.cpp) over
    every model, law, side condition, Dirichlet data, a solid body, the three
    lattice-speed modes, the tangent runs and the rejected inputs;
  * tests/sanitize/abi_main.cpp -- the library's host-side checks
    (csrc/lbrs_host.cpp: parameter validation and the node codes of solid
    bodies) over random and edge-case parameters and random bodies.
Also: the OpenMP timing build of the oracle gives the serial build's bits."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1504_07034_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]


def _build_and_run(tmp_path, name, sources, extra=()):
    exe = str(tmp_path / name)
    subprocess.check_call(["g++", *SAN, *extra, *sources, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "clean" in r.stdout
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_sanitizers(tmp_path):
    _build_and_run(tmp_path, "oracle_main", [os.path.join(ROOT, "tests", "sanitize", "oracle_main.cpp")])


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_checks_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1504_07034_amd", "csrc")
    _build_and_run(tmp_path, "abi_main",
                   [os.path.join(ROOT, "tests", "sanitize", "abi_main.cpp"),
                    os.path.join(csrc, "lbrs_host.cpp")],
                   extra=["-I", os.path.join(ROOT, "include"), "-I", csrc])


def test_openmp_build_gives_the_serial_bits():
    """The timing build (OpenMP over cells, -O3 -march=native, no contraction)
    and the serial build agree bit for bit: per-step speeds on the four-quadrant
    problem, the explosion between walls, and the 1D tube."""
    cases = []
    w = wl.riemann2d(48)
    cases.append((oracle.Problem(model=w.model, nx=w.nx, ny=w.ny, domain=w.domain), w.W, 0.1))
    w = wl.explosion(40, t_end=0.05)
    cases.append((oracle.Problem(model=w.model, nx=w.nx, ny=w.ny, domain=w.domain, omega=1.5,
                                 sides=(oracle.WALL, oracle.WALL, oracle.PERIODIC, oracle.PERIODIC)),
                  w.W, 0.05))
    w = wl.sod(400)
    cases.append((oracle.Problem(model=w.model, nx=w.nx, domain=w.domain), w.W, 0.2))
    try:
        for P, W, t_end in cases:
            oracle.use("serial")
            a = oracle.run(P, oracle.prim_to_cons(P, W), t_end=t_end)
            assert oracle.use("omp", 4) == 4
            b = oracle.run(P, oracle.prim_to_cons(P, W), t_end=t_end)
            assert a.status == 0 and a.nsteps == b.nsteps and np.array_equal(a.dt, b.dt)
            assert np.array_equal(a.U, b.U)
    finally:
        oracle.use("serial")
