"""The library's host linear algebra (csrc/hostla.cpp: the set-up eigensolver -- Householder
tridiagonalization and QL with threaded back-transformation -- and the small Cholesky factor and
triangular inverse) built for the CPU with AddressSanitizer and UndefinedBehaviorSanitizer and run
over sizes that take the serial and the threaded branches and over degenerate spectra (zero,
identity, repeated and clustered eigenvalues).  Any sanitizer report fails the test, and so does
an inaccurate decomposition."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2111_11473_amd", "csrc")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("san") / "hostla_san")
    flags = ["-O1", "-g", "-std=c++17", "-pthread", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    r = subprocess.run([gxx, *flags, "-I", CSRC, os.path.join(HERE, "hostla_main.cpp"),
                        os.path.join(CSRC, "hostla.cpp"), "-o", out], capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in r.stderr.lower() and "cannot find" in r.stderr.lower():
        pytest.skip("sanitizer runtime not installed")
    assert r.returncode == 0, r.stderr
    return out


def _run(exe, kind, n):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe, kind, str(n)], capture_output=True, text=True, env=env, timeout=300)
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (kind, n, r.returncode, r.stderr[-2000:])
    return [float(x) for x in r.stdout.split()]


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 65, 130, 257])
@pytest.mark.parametrize("kind", ["random", "diagonal", "identity", "rank1", "zero", "clustered"])
def test_eigensolver_under_sanitizers(exe, kind, n):
    res, orth = _run(exe, kind, n)
    assert res < 1e-12 and orth < 1e-12, (kind, n, res, orth)


@pytest.mark.parametrize("n", [1, 2, 5, 64, 100])
def test_cholesky_under_sanitizers(exe, n):
    err, inv = _run(exe, "spd", n)
    assert err < 1e-13 and inv < 1e-12, (n, err, inv)
