"""Helpers to run the CPU harness of the device code (tests/cpu_harness)."""
import os
import subprocess
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpu_harness", "emu.cpp")
_EXE = {}


def emu_exe(line_vec=True):
    """The harness binary; line_vec=False compiles out the line passes'
    16-byte fast path."""
    if line_vec not in _EXE:
        d = tempfile.mkdtemp(prefix="ch_emu_")
        exe = os.path.join(d, "emu")
        subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                        f"-DCH_LINE_VEC={1 if line_vec else 0}", "-o", exe, SRC], check=True)
        _EXE[line_vec] = exe
    return _EXE[line_vec]


def pack(arrays):
    return np.concatenate([np.ascontiguousarray(a, dtype=np.float64).ravel() for a in arrays])


def run_emu(boxes, dt, nsteps, prec=0, kappa=4.0, eps=1e-6, solve=0, x_rows=0, seg=0,
            waves=0, z_chunk=0, mode=0, x_general=0, line_vec=True):
    """boxes: list of dicts with C, u, v, w, h, Cn, Pe, bc.  Returns (list of
    C arrays, masses, plan dict)."""
    with tempfile.TemporaryDirectory() as d:
        with open(os.path.join(d, "params.txt"), "w") as f:
            f.write(f"{len(boxes)} {prec} {kappa!r} {eps!r} {solve} {x_rows} {seg} {waves} "
                    f"{z_chunk} {dt!r} {nsteps} {mode} {x_general}\n")
            for b in boxes:
                nz, ny, nx = b["C"].shape
                bc = b.get("bc", (0, 0, 0))
                f.write(f"{nx} {ny} {nz} {b['h']!r} {b['Cn']!r} {b['Pe']!r} "
                        f"{bc[0]} {bc[1]} {bc[2]}\n")
        for name in ("C", "u", "v", "w"):
            pack([b[name] for b in boxes]).tofile(os.path.join(d, name + ".bin"))
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([emu_exe(line_vec), os.path.join(d, "params.txt"), d, d], env=env,
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"emu failed ({r.returncode}):\n{r.stderr[-4000:]}")
        flat = np.fromfile(os.path.join(d, "C.bin"), dtype=np.float64)
        masses = [float(x) for x in open(os.path.join(d, "mass.txt")).read().split()]
        p = open(os.path.join(d, "plan.txt")).read().split()
        plan = dict(x_rows=int(p[0]), seg=int(p[1]), yz_threads=int(p[2]), tw_max=int(p[3]),
                    acc64=int(p[4]), ntask=[int(x) for x in p[5:8]],
                    lds=[int(x) for x in p[8:11]], z_chunk=int(p[11]), xrow=int(p[12]), nxl=int(p[13]),
                    xrm=[int(x) for x in p[14:17] if int(x) >= 0],
                    nth=[int(x) for x in p[17:20] if int(x) >= 0])
    out, o = [], 0
    for b in boxes:
        n = b["C"].size
        out.append(flat[o:o + n].reshape(b["C"].shape))
        o += n
    return out, masses, plan


_STENCIL_EXE = None


def lib_stencils(kind, s, targets):
    """The library's 1-D transfer stencils (ch_plan.h, built for the host
    with sanitizers): (idx [m,4] int, w [m,4] float64), or None when the
    library refuses the axis."""
    global _STENCIL_EXE
    if _STENCIL_EXE is None:
        d = tempfile.mkdtemp(prefix="ch_stencil_")
        exe = os.path.join(d, "stencil_dump")
        subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", exe,
                        os.path.join(ROOT, "tests", "cpu_harness", "stencil_dump.cpp")],
                       check=True)
        _STENCIL_EXE = exe
    s = np.asarray(s, dtype=np.float64)
    t = np.atleast_1d(np.asarray(targets, dtype=np.float64))
    text = f"{int(kind)} {s.size}\n" + " ".join(repr(float(x)) for x in s) + \
        f"\n{t.size}\n" + " ".join(repr(float(x)) for x in t) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([_STENCIL_EXE], input=text, capture_output=True, text=True, env=env)
    if r.returncode != 0:
        raise RuntimeError(f"stencil_dump failed ({r.returncode}):\n{r.stderr[-4000:]}")
    if r.stdout.strip() == "FAIL":
        return None
    rows = [line.split() for line in r.stdout.strip().splitlines()]
    idx = np.array([[int(x) for x in row[:4]] for row in rows], dtype=np.int64)
    w = np.array([[float(x) for x in row[4:]] for row in rows], dtype=np.float64)
    return idx, w
