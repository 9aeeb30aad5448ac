"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The library's host C++ (mesh half-edges, quadrature, laydown, tracking, links, volumes,
  segment packing, coarse-mesh surfaces, the DFEM-SN schedule, the HFEM set-up) is built
  with both sanitizers on its host compilation and runs the host-only library tests
  (test_library_host.py) in a child process that preloads clang's sanitizer runtime.
* The C oracles (planar MOC, DGMOC, DFEM-SN) are built with gcc's sanitizers and run
  their pin tests in a child process that preloads gcc's libasan.
* A heap overflow planted in a separate small library, built each way, shows that the
  sanitizers fire in this set-up (the child exits non-zero with an AddressSanitizer
  report).
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

PLANTED = r'''
#include <stdlib.h>
#ifdef __cplusplus
extern "C"
#endif
int planted(int n) {
    int *a = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i <= n; ++i) a[i] = i;   /* one past the end */
    int s = a[n - 1];
    free(a);
    return s;
}
'''


def _gcc_asan():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    path = r.stdout.strip()
    if not os.path.isabs(path):
        pytest.skip("gcc's libasan not found")
    return path


def _run(code, preload, timeout=900):
    env = dict(ENV, LD_PRELOAD=preload)
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=timeout)


def _clean(r):
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]


def test_planted_overflow_is_caught_by_both_builds():
    from paper_2607_01591_amd import build as B
    with tempfile.TemporaryDirectory() as d:
        src_c = os.path.join(d, "planted.c")
        open(src_c, "w").write(PLANTED)
        so_gcc = os.path.join(d, "planted_gcc.so")
        subprocess.check_call(["gcc", "-O1", "-g", "-fPIC", "-shared", "-fsanitize=address,undefined",
                               "-fno-omit-frame-pointer", "-o", so_gcc, src_c])
        src_cpp = os.path.join(d, "planted.cpp")
        open(src_cpp, "w").write(PLANTED)
        obj = os.path.join(d, "planted.o")
        subprocess.check_call([B.HIPCC, "-x", "hip", "--offload-arch=gfx950", "-fPIC"] + B.SAN_FLAGS +
                              ["-c", src_cpp, "-o", obj])
        so_clang = os.path.join(d, "planted_clang.so")
        subprocess.check_call([B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", so_clang, obj])
        for so, rt in ((so_gcc, _gcc_asan()), (so_clang, B.sanitizer_runtime())):
            r = _run(f"import ctypes; print(ctypes.CDLL({so!r}).planted(8))", rt, timeout=120)
            assert r.returncode != 0 and "AddressSanitizer" in r.stderr, (so, r.returncode, r.stderr[-2000:])


def test_library_host_code_under_sanitizers():
    from paper_2607_01591_amd import build as B
    with tempfile.TemporaryDirectory() as d:
        so = B.build_sanitized(d)
        code = ("import sys; sys.path.insert(0, '.')\n"
                "from paper_2607_01591_amd import moc\n"
                f"moc.LIB_PATH = {so!r}\n"
                "import pytest\n"
                "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', 'tests/test_library_host.py']))\n")
        _clean(_run(code, B.sanitizer_runtime()))


def test_oracles_under_sanitizers():
    from oracle import dg_oracle, oracle, sn_oracle
    with tempfile.TemporaryDirectory() as d:
        paths = {m: m.build_sanitized(os.path.join(d, os.path.basename(m._SO))) for m in (oracle, dg_oracle, sn_oracle)}
        code = ("import sys; sys.path.insert(0, '.')\n"
                "import oracle.oracle as O, oracle.dg_oracle as D, oracle.sn_oracle as S\n"
                f"O._SO = {paths[oracle]!r}; D._SO = {paths[dg_oracle]!r}; S._SO = {paths[sn_oracle]!r}\n"
                "import pytest\n"
                "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', 'tests/test_oracle.py', "
                "'tests/test_dgmoc_oracle.py', 'tests/test_dfem_oracle.py', "
                "'-k', 'not threads_change_nothing']))\n")
        _clean(_run(code, _gcc_asan()))
