"""Sanitizer builds on the host (CPU only, no GPU needed).

* The FP64 oracle built with AddressSanitizer + UBSan gives bitwise the results
  of its normal build on pair sets, forces (every model, a triclinic box), a
  subset of rows and a short trajectory, with no sanitizer report.
* libnb built with ASan + UBSan on its host code (the device code as usual):
  a C++ driver (sanitize_host_driver.cpp) runs every entry point that needs no
  GPU -- parameter validation and arena sizing over the parameter space, status
  strings, NULL-handle error paths -- with no sanitizer report.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_runtime(name):
    return subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()


def _clean(out):
    return "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out


def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-fPIC", "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "oracle.c"), "-o", lib, "-lm"])
    script = textwrap.dedent(f"""
        import ctypes, sys
        import numpy as np
        sys.path.insert(0, {ROOT!r})
        import oracle
        from paper_1506_00716_amd import inputs

        def run():
            out = []
            s = inputs.small_rf()
            out.append(oracle.pairs(s.x, s.box, s.model.r_list, nthreads=1))
            out += list(oracle.forces(s, nthreads=1))
            m = inputs.Model(r_cut=0.9, r_list=1.0, coulomb="ewald", ewald_beta=3.12, lj="lb")
            t = inputs.random_triclinic_system(300, (2.6, 2.4, 2.5), (0.9, -0.6, 0.7), 3, m)
            out.append(oracle.pairs(t.x, t.box, 1.0, nthreads=1, box_off=t.box_off))
            out += list(oracle.forces(t, nthreads=1))
            out += list(oracle.forces_subset(t, np.array([5, 0, 299, 5], dtype=np.int32), nthreads=1))
            d = inputs.tiny_random_system(200, (3.0, 3.1, 3.2), 4, inputs.Model(r_cut=0.9, r_list=1.0, coulomb="rf"),
                                          min_dist=0.3)
            v = inputs.maxwell_velocities(np.random.default_rng(4), d.mass, 300.0)
            out += list(oracle.md(d, d.x, v, 0.002, 5, nthreads=1))
            return out

        ref = run()
        oracle._lib = oracle.configure(ctypes.CDLL({lib!r}))
        san = run()
        assert len(ref) == len(san)
        for a, b in zip(ref, san):
            assert np.array_equal(np.asarray(a), np.asarray(b))
        print("oracle under sanitizers: identical results")
    """)
    env = dict(os.environ, LD_PRELOAD=_gcc_runtime("libasan.so") + ":" + _gcc_runtime("libubsan.so"),
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert _clean(out), out[-4000:]
    assert "identical results" in r.stdout


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    from paper_1506_00716_amd import build as B
    flags = [f for f in B.COMMON if f != "-O3"] + ["-O1", "-g", "-Xarch_host", "-fsanitize=address",
                                                   "-Xarch_host", "-fsanitize=undefined",
                                                   "-Xarch_host", "-fno-omit-frame-pointer",
                                                   "-Xarch_device", "-O3", "-Wno-unused-value"]
    procs, objs = [], []
    for src, extra in B.SOURCES.items():
        obj = str(tmp_path / src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([B.hipcc(), *flags, *extra, "-c", os.path.join(B.CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate(timeout=900)
        assert p.returncode == 0, out[-4000:]
    lib = str(tmp_path / "libnb_san.so")
    subprocess.check_call([B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-Xarch_host",
                           "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *objs, *B.LINK, "-o", lib])
    drv = str(tmp_path / "host_driver")
    clangxx = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++")
    subprocess.check_call([clangxx, "-std=c++17", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           os.path.join(ROOT, "tests", "sanitize_host_driver.cpp"), "-L", str(tmp_path),
                           "-lnb_san", "-Wl,-rpath," + str(tmp_path), "-o", drv])
    r = subprocess.run([drv], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"), capture_output=True, text=True,
                       timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert _clean(out), out[-4000:]
    assert "0 failure(s)" in r.stdout
