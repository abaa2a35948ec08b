"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): libgwd is
built with both sanitizers on its host code (paper_2201_11133_amd/build_asan.py; the gfx950 device
code is unchanged) and the CPU tests of test_abi.py (argument checks, sizes, error paths, the
allocation-free trigger entry's limits) run against it in a child process that has the sanitizer
runtime preloaded. Any sanitizer report, or a failing test, fails this test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(900)
def test_abi_cpu_tests_under_host_sanitizers(tmp_path):
    from paper_2201_11133_amd import build_asan
    runtime = build_asan.runtime_path()
    if not runtime or not os.path.exists(runtime):
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    lib = build_asan.build()
    script = "\n".join([
        "import sys",
        f"sys.path.insert(0, {ROOT!r})",
        "import paper_2201_11133_amd.gwd as g",
        f"g.lib = g._load({lib!r})",
        "import pytest",
        f"sys.exit(pytest.main([{os.path.join(ROOT, 'tests', 'test_abi.py')!r}, '-m', 'not gpu', '-q', "
        "'-p', 'no:cacheprovider', '-x']))",
    ])
    pre = os.environ.get("LD_PRELOAD", "")
    env = dict(os.environ,
               LD_PRELOAD=runtime + (":" + pre if pre else ""),
               ASAN_OPTIONS=f"detect_leaks=0:halt_on_error=1:log_path={tmp_path}/asan",
               UBSAN_OPTIONS=f"halt_on_error=1:print_stacktrace=1:log_path={tmp_path}/ubsan")
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=600)
    reports = {p: open(p).read() for p in glob.glob(str(tmp_path / "*san*"))}
    print(r.stdout[-2000:])
    assert not reports, "\n".join(v[:3000] for v in reports.values())
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
