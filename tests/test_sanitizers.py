"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer runs (no GPU needed).

- the oracle's C code (gcc), driven by tests/sanitize/oracle_driver.c over every function it
  exports, on small sizes;
- the library's host code: every library source compiled with hipcc with the sanitizers on the
  host pass only (the device code is built as usual and never runs here), linked with the driver
  tests/sanitize/host_driver.cpp, which exercises the host-only queries over many shapes, every
  entry point's refusal of NULL arguments and context creation on a device that does not exist.

The library build is kept in the system's temporary directory under the hash of its sources,
so only the first run after a source change pays for it (about a minute).
"""
import hashlib
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_18396_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc absent")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_san")
        _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
              os.path.join(ROOT, "oracle", "pimm_oracle.c"), os.path.join(SAN, "oracle_driver.c"),
              "-o", exe, "-lm"])
        out = _run([exe], env=ENV, timeout=300)
    assert out.strip().splitlines()[-1].startswith("ok ")


def _library_build():
    """Host-sanitized objects of every library source (cached by the sources' hash)."""
    from paper_2305_18396_amd import build as b

    srcs = [os.path.join(CSRC, s) for s in b.HIP_SOURCES]
    headers = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h"))
    h = hashlib.sha256()
    for f in srcs + headers + [os.path.join(CSRC, s) for s in b.HOST_SOURCES] + \
            [os.path.join(INCLUDE, "pimm.h")]:
        h.update(open(f, "rb").read())
    out = os.path.join(tempfile.gettempdir(), "pimm_sanitize_" + h.hexdigest()[:16])
    done = os.path.join(out, "objs.txt")
    if os.path.exists(done):
        return [os.path.join(out, o) for o in open(done).read().split()]
    os.makedirs(out, exist_ok=True)
    flags = [f for f in b.HIPCC_FLAGS if f != "-O3"] + ["-O1"]
    # The sanitizers go to the host pass only.
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    procs, objs = [], []
    for s in srcs:
        o = os.path.join(out, os.path.basename(s) + ".o")
        procs.append(subprocess.Popen([b.hipcc(), *flags, *san, "-I" + INCLUDE, "-I" + CSRC, "-c", s,
                                       "-o", o], stdout=subprocess.PIPE, stderr=subprocess.PIPE))
        objs.append(o)
    for s in b.HOST_SOURCES:
        o = os.path.join(out, s + ".o")
        _run(["g++", "-O1", "-g", "-fPIC", "-std=c++17", "-fsanitize=address,undefined",
              "-fno-omit-frame-pointer", "-I" + INCLUDE, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err.decode()[-3000:]
    with open(done, "w") as fh:
        fh.write(" ".join(os.path.basename(o) for o in objs))
    return objs


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc absent")
def test_library_host_code_under_sanitizers():
    clang = _clang()
    if clang is None:
        pytest.skip("clang++ absent")
    objs = _library_build()
    with tempfile.TemporaryDirectory() as d:
        drv = os.path.join(d, "driver.o")
        exe = os.path.join(d, "host_san")
        _run([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
              "-fno-omit-frame-pointer", "-I" + INCLUDE, "-c", os.path.join(SAN, "host_driver.cpp"),
              "-o", drv])
        _run([clang, "-fsanitize=address,undefined", drv, *objs, "-L/opt/rocm/lib", "-lamdhip64",
              "-lquadmath", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
        out = _run([exe], env=ENV, timeout=600)
    assert out.strip().splitlines()[-1].startswith("ok ")
