"""The host setup code (coarsening, interpolation, Galerkin products,
composite sets, batched layouts, 16-bit index compression, padding 0 with
empty coarse levels, transposed hierarchies for the adjoint) built with
AddressSanitizer and UndefinedBehaviorSanitizer and run over every setup
variant by a small C++ driver (tests/host/setup_check.cpp).  CPU only."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_setup_under_asan_ubsan(tmp_path):
    exe = tmp_path / "setup_check"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-pthread",
           os.path.join(ROOT, "tests", "host", "setup_check.cpp"),
           os.path.join(ROOT, "paper_1906_10575_amd", "csrc", "setup.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", AMGDD_THREADS="4")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "36 setups, 0 failed" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_sliced_ell_packing_matches_the_device_walk(tmp_path):
    """Sliced-ELL packing with one, two or four entries per lane and step, every lane count, ragged and
    empty rows: the addresses each lane of the device mat-vec reads give the
    row's entries in the documented accumulation order (under ASan/UBSan)."""
    exe = tmp_path / "sell_layout_check"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-pthread",
           os.path.join(ROOT, "tests", "host", "sell_layout_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=dict(os.environ, AMGDD_THREADS="4"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "450 layouts, 0 failed" in r.stdout
