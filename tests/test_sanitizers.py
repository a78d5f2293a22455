"""Sanitizer runs on the CPU (no GPU involved).

* The oracle, built with AddressSanitizer and UndefinedBehaviorSanitizer
  (gcc), runs its pin tests.
* The library's host code, built with the same sanitizers on the host side
  only (hipcc; the device code is compiled as usual), runs the C-ABI
  argument-validation tests: every entry point's checks, on NULL handles and
  invalid sizes, execute under the sanitizers without touching a device.

Each run is a subprocess with the sanitizer runtime preloaded and any report
fatal.  The sanitized builds are cached under paper_2208_01339_amd/_build/san
and rebuilt when their sources change.
"""
import glob
import os
import subprocess
import sys

import pytest

from conftest import ROOT

SAN_DIR = os.path.join(ROOT, "paper_2208_01339_amd", "_build", "san")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _stale(out, deps):
    return not os.path.exists(out) or any(os.path.getmtime(d) > os.path.getmtime(out) for d in deps)


def _env(extra):
    env = dict(os.environ)
    env.update(extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


def _pytest(env, args, timeout):
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *args], cwd=ROOT,
                          env=env, capture_output=True, text=True, timeout=timeout)


def _gcc_runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip("gcc has no %s here" % name)
    return p


def test_oracle_under_asan_ubsan():
    src = os.path.join(ROOT, "oracle", "ppcg_oracle.c")
    so = os.path.join(SAN_DIR, "liboracle_san.so")
    os.makedirs(SAN_DIR, exist_ok=True)
    if _stale(so, [src]):
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                               "-o", so, src, "-lm"])
    env = _env({"PPCG_ORACLE_LIB": so,
                "LD_PRELOAD": _gcc_runtime("libasan.so") + " " + _gcc_runtime("libubsan.so")})
    probe = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.lib()._name)"], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0 and probe.stdout.strip() == so, probe.stdout + probe.stderr
    files = ["tests/test_oracle_pins.py", "tests/test_oracle_dfn.py", "tests/test_oracle_lowrank.py",
             "tests/test_oracle_mlp.py"]
    r = _pytest(env, files + ["-k", "not omp"], 1200)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]


def test_library_host_code_under_asan_ubsan():
    from paper_2208_01339_amd import build as hb

    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts or not os.path.exists(HIPCC):
        pytest.skip("no hipcc / clang ASan runtime")
    objdir = os.path.join(ROOT, "paper_2208_01339_amd", "_build")
    plain = [os.path.join(objdir, f + ".o") for f in ("pp_batch.hip", "pp_mlp.hip")]
    if any(_stale(o, hb.DEPS) for o in plain):
        hb.build(verbose=False)
    os.makedirs(SAN_DIR, exist_ok=True)
    flags = [f for f in hb.FLAGS if f != "-shared"]
    flags = [f for f in flags if f != "-O3"] + ["-O1", "-g"]
    for opt in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                "-fno-omit-frame-pointer"):
        flags += ["-Xarch_host", opt]  # host code only
    objs, procs = [], []
    for name in ("pp_lib.hip", "pp_noalloc.hip"):
        obj = os.path.join(SAN_DIR, name + ".o")
        objs.append(obj)
        if _stale(obj, hb.DEPS + [os.path.join(os.path.dirname(hb.SRC[0]), "pp_noalloc.hip")]):
            procs.append(subprocess.Popen([HIPCC, *flags, "-c", "-o", obj, os.path.join(os.path.dirname(hb.SRC[0]),
                                                                                          name)]))
    assert all(p.wait() == 0 for p in procs)
    so = os.path.join(SAN_DIR, "libppcg_san.so")
    if _stale(so, objs + plain):
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", so, *objs, *plain])
    env = _env({"PPCG_LIB": so, "LD_PRELOAD": rts[-1]})
    r = _pytest(env, ["tests/test_abi.py", "-k", "not refuses_missing"], 600)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "passed" in r.stdout
