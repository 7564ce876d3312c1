"""Host checks of the WENO5 face arithmetic the x pass runs (the same
header compiled for the CPU): the increment is odd in the differences bit for
bit, the downwind reading of a stencil is the centre minus the increment of
the reversed forward differences bit for bit, the shared-difference flux
u C_up + |u| inc matches u times the value-based upwinded face value to
rounding, the fourth difference from first differences matches the
(1, -4, 6, -4, 1) stencil (exactly on integer data), and the face value
matches the Jiang-Shu formula written out plainly (candidates, smoothness
indicators, normalised weights) to 1e-12 in double precision.  Sec. 2.2 (WENO5
advection) and eq-a3d (fourth differences)."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpu_harness", "weno_check.cpp")


def test_weno_face_arithmetic_identities():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "weno_check")
        subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-o", exe, SRC], check=True)
        r = subprocess.run([exe], capture_output=True, text=True,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    print(r.stdout[-2000:])
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), \
        r.stdout[-2000:] + r.stderr[-2000:]
