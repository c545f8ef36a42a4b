"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle (gcc, -fsanitize=address,undefined) runs its pins, and the host side of libpt
(hipcc, host-only sanitizers: scene build, binned-SAH BVH, four-wide collapse, node
quantization, C-ABI argument checks, batch bookkeeping) runs the host tests of the C ABI
and of the serving loop, each in a child process with the compiler's ASan runtime
preloaded.  A report from either sanitizer ends its child process with a failure."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"sanitizer runtime not found ({' '.join(cmd)})")
    return path


def _run_under(preload, env_extra, tests, tmp_path):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = preload
    log = str(tmp_path / "san")
    env["ASAN_OPTIONS"] = f"detect_leaks=0:log_path={log}"    # the interpreter itself holds memory at exit
    env["UBSAN_OPTIONS"] = f"halt_on_error=1:print_stacktrace=1:log_path={log}"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = ""
    for f in sorted(os.listdir(tmp_path)):
        if f.startswith("san."):
            with open(tmp_path / f) as fh:
                reports += fh.read()
    assert r.returncode == 0 and not reports, (r.stdout[-3000:] + r.stderr[-3000:] + reports[:6000])
    return r.stdout


def test_oracle_pins_under_asan_ubsan(tmp_path):
    from oracle.build import build_sanitized
    lib = build_sanitized()
    asan = _runtime(["gcc", "-print-file-name=libasan.so"])
    out = _run_under(asan, {"PT_ORACLE_LIB": lib},
                     ["tests/test_oracle_pins.py", "tests/test_oracle_golden.py", "-k",
                      "not unbiased and not ggx_weight_mean"], tmp_path)
    assert " passed" in out


def test_libpt_host_code_under_asan_ubsan(tmp_path):
    from paper_2310_07182_amd import build as pb
    lib = pb.build(sanitize=True)
    asan = _runtime(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"])
    out = _run_under(asan, {"PT_LIB": lib}, ["tests/test_capi_host.py", "tests/test_serve_host.py"], tmp_path)
    assert " passed" in out
