"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle's C source is compiled with gcc -fsanitize=address,undefined
(errors abort, no recovery) and the pin battery of the mutation tests is run
against that build in a child process that preloads the ASan runtime.  Any
out-of-bounds access, use after free or undefined arithmetic in the oracle
ends the child with a sanitizer report; the pins must still all pass.
"""
import os
import subprocess
import sys
import textwrap

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-fPIC", "-shared", "-std=c99", "-Wall", "-Wextra"]


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def _run_sanitized_battery(source, tmp_path):
    """Build `source` with the sanitizers and run the pin battery against it
    in a child process; returns (exit code, stdout, stderr)."""
    runtime = _asan_runtime()
    if runtime is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    src = os.path.join(str(tmp_path), "trt_oracle_san.c")
    lib = os.path.join(str(tmp_path), "libtrt_oracle_san.so")
    with open(src, "w") as fh:
        fh.write(source)
    subprocess.run(["gcc", *SAN_FLAGS, src, "-o", lib, "-lm"], check=True)
    child = textwrap.dedent("""
        import sys
        sys.path[:0] = [%r, %r]
        import oracle
        import test_oracle_mutations as mut
        failed = mut._battery(oracle.Oracle(%r))
        print("FAILED_PINS", failed, flush=True)
        sys.exit(1 if failed else 0)
    """ % (ROOT, HERE, lib))
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=97"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([sys.executable, "-c", child], capture_output=True, text=True, env=env,
                       timeout=900)
    return r.returncode, r.stdout, r.stderr


def test_pin_battery_passes_under_address_and_ub_sanitizers(tmp_path):
    rc, out, err = _run_sanitized_battery(oracle.source_text(), tmp_path)
    report = out[-4000:] + err[-4000:]
    assert "AddressSanitizer" not in err, report
    assert "runtime error" not in err, report
    assert rc == 0, report
    assert "FAILED_PINS []" in out, report


def test_sanitized_run_reports_a_planted_out_of_bounds_read(tmp_path):
    """The check above can fail: an oracle whose gradient reads one element
    past the end of its Phi array (the last node's x + 1 neighbour without
    the periodic wrap) is stopped by AddressSanitizer."""
    good = "0.5 * (phix[(long)y * nx + wrap(x + 1, nx)] - phix[(long)y * nx + wrap(x - 1, nx)])"
    bad = "0.5 * (phix[(long)y * nx + (x + 1)] - phix[(long)y * nx + wrap(x - 1, nx)])"
    src = oracle.source_text()
    assert src.count(good) == 1
    rc, out, err = _run_sanitized_battery(src.replace(good, bad), tmp_path)
    assert rc == 97 and "heap-buffer-overflow" in err, (out[-2000:], err[-2000:])
