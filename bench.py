"""Benchmark of the Cahn-Hilliard update on one MI355X.

Workload: the 256^3 periodic box with 64 tanh drops (radii 6-16 h) in a
frozen divergence-free k^-5/3 velocity field (1 <= k <= 16, rms 1),
Cn = h, Pe = 0.9/Cn, dt = 1e-4.  Inputs are seeded and synthetic and are
resident in HBM before the timed region starts.

A step is one full RK3 step (3 substages x {x pass, y solve, z solve}).
`value` is the FP32 throughput in grid-point updates per second (Gpts/s);
the FP64 throughput, the FP32-vs-FP64 error after --acc-steps steps (1000
by default, whatever --steps is), the roofline of the dominant kernel (the
x pass, against HBM and against vector instruction issue) and the FP64 CPU
oracle's throughput on a bounded sample of the same workload are reported
on the same JSON line, with the other workloads' lines.

    python bench.py [--steps K] [--warmup W]
    python bench.py --counter-probe [fp64]    # 2 FP32 (FP64) steps + one 256 MiB device
                                       # copy, for rocprofv3 counter runs
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, vendor figure
# Vector FMA rate without packed FP32 (which this library does not emit):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz, the same in FP32 and FP64.
VALU_PEAK_TFLOPS = 78.6
# MI355X's published FP32 vector peak (packed FP32 math)
VALU_PEAK_PUBLISHED_FP32_TFLOPS = 157.3
# Vector instruction issue: a SIMD takes one wave64 VALU instruction every 4
# cycles (16 lanes per cycle): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# lane-instructions per second, whatever the instruction.
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9
# A device-to-device copy of 4 GiB or more on MI355X (torch copy, read +
# write bytes over time): the HBM rate a streaming kernel can reach.
COPY_GBS = 4900.0
METRIC = ("CH grid-point updates/s (Gpts/s) FP32 & batched vs FP64 at stated error; "
          "%HBM peak")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pass_x_256cube_fp32_traffic.md")
TRAFFIC_FILE_LARGE = os.path.join(ROOT, "profiles", "k_pass_x_1536cube_fp32_traffic.md")
SQ_FILE = os.path.join(ROOT, "profiles", "k_passes_256cube_fp32_sq_counters.md")
SQ_FILE_LARGE = os.path.join(ROOT, "profiles", "k_passes_1536cube_fp32_sq_counters.md")
X_SOURCES = ("ch_device.h", "ch_kernels.hip", "ch_plan.h")
DROPS_DEF = ("face-connected cells with C >= 1/2 (periodic axes wrap, walls do not connect), "
             "V = h^3 cells, (4 pi/3)(D/2)^3 = V, H = box height")


def progress(msg):
    """One line per finished section on stderr (long runs stay visibly alive)."""
    print(f"[bench] {msg} ({time.perf_counter() - _T0:.0f} s)", file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def x_pass_flops_per_point():
    """Algorithmic flops of one x-pass launch per grid point (fused
    multiply-add = 2, add / multiply / reciprocal = 1):
      WENO5 face value times velocity, 55 per face, one face per cell and
      direction: 165;  flux divergence and 1/h: 6;  psi'(C) and its 7-point
      Laplacian: 13;  three fourth differences and their sum: 26;  E and the
      RHS: 7;  the x-line recurrences (forward 5, backward 4): 9."""
    return 165 + 6 + 13 + 26 + 7 + 9


def x_pass_bytes_per_point(s):
    """Algorithmic HBM bytes per grid point of one x-pass launch, averaged over
    the three substages: reads C, u, v, w (+ the old E in substages 2 and 3),
    writes the RHS q (+ the new E in substages 1 and 2): 6s, 7s, 6s."""
    return (6 + 7 + 6) / 3.0 * s


def step_bytes_per_point(s):
    """Algorithmic bytes per point of a whole RK3 step: 34 s (three passes of
    11, 12, 11 element accesses)."""
    return 34.0 * s


def x_source_hash():
    h = hashlib.sha256()
    for f in X_SOURCES:
        with open(os.path.join(ROOT, "paper_2105_01865_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_value(path, key):
    """The number on the `key:` line of a committed counter summary, if the
    summary was taken on the current kernel sources; otherwise None."""
    try:
        text = open(path).read()
    except OSError:
        return None
    src = re.search(r"^source-hash:\s*(\w+)", text, re.M)
    val = re.search(r"^" + re.escape(key) + r":\s*([0-9.eE+]+)", text, re.M)
    if not src or not val or src.group(1) != x_source_hash():
        return None
    return float(val.group(1))


def measured_traffic(path=None):
    """HBM bytes per x-pass launch from a committed counter summary (the
    256^3 one unless `path` names another), or None."""
    return profile_value(path or TRAFFIC_FILE, "traffic-bytes-per-launch")


def issue_view(avg_us, path=None):
    """The x pass against vector instruction issue: its VALU lane-instructions
    per launch (counted, from a committed summary for the current sources)
    over its average launch time, as a fraction of VALU_ISSUE_PEAK; None
    without a matching summary."""
    n = profile_value(path or SQ_FILE, "x-pass-valu-lane-instructions-per-launch")
    if n is None:
        return None
    rate = n / (avg_us * 1e-6)
    return {"valu_lane_instructions_per_launch": n,
            "achieved_lane_instructions_per_s": round(rate / 1e12, 3),
            "peak_lane_instructions_per_s": round(VALU_ISSUE_PEAK / 1e12, 3),
            "unit": "10^12 lane-instructions/s", "frac": round(rate / VALU_ISSUE_PEAK, 4)}


def limiter(issue, traffic, avg_us):
    """The limit the x pass runs nearer to: vector instruction issue (the
    fraction of VALU_ISSUE_PEAK in `issue`) or HBM (its counted traffic per
    launch at COPY_GBS); None without both counts."""
    if not issue or not traffic:
        return None
    hbm = traffic / (avg_us * 1e-6) / 1e9 / COPY_GBS
    return {"limiter": "valu_issue" if issue["frac"] >= hbm else "hbm",
            "issue_frac": issue["frac"], "hbm_frac_of_copy_rate": round(hbm, 4),
            "copy_gbs": COPY_GBS}


def x_roofline(avg_us, points, es, traffic=None, kernel="k_pass_x"):
    """The x pass (explicit terms, RHS and x solve) against HBM: algorithmic
    bytes of one launch (x_pass_bytes_per_point x points) over its average
    launch time from HIP events; `traffic` is the counter-measured HBM bytes
    of one launch, when a summary for the current sources exists."""
    nbytes = x_pass_bytes_per_point(es) * points
    gbs = nbytes / (avg_us * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic, "algorithmic_bytes_per_launch": nbytes,
            "avg_launch_us": round(avg_us, 2)}


def step_hbm_frac(points, es, ms_per_step, extra_bytes=0.0):
    """Whole-step algorithmic bytes (34 element accesses per point, plus any
    transfer bytes) over the step time, as a fraction of HBM peak."""
    return round((step_bytes_per_point(es) * points + extra_bytes) /
                 (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)


def dh_histogram(cells, h, H, nbins=12):
    """PDF of D/H over drops (D the equivalent-sphere diameter of the drop's
    volume h^3 cells): equal bins from 0 to the largest D/H."""
    import numpy as np
    if len(cells) == 0:
        return None
    dh = np.cbrt(6.0 * np.asarray(cells, dtype=np.float64) * h ** 3 / np.pi) / H
    top = float(dh.max()) * 1.0001
    counts, edges = np.histogram(dh, bins=nbins, range=(0.0, top))
    width = edges[1] - edges[0]
    return {"drops": int(len(dh)), "edges": [round(float(e), 5) for e in edges],
            "counts": [int(c) for c in counts],
            "pdf": [round(float(c) / (len(dh) * width), 4) for c in counts],
            "min": float(dh.min()), "median": float(np.median(dh)), "max": float(dh.max())}


def fp32_errors(C32, C64, m32, m64, drops32, drops64, h, H, steps):
    """FP32 against FP64 after `steps` steps from the same field: relative
    L2(C), the FP64-summed mass drift of each, the drop-volume error
    |V32 - V64| / V64 with V = h^3 #{C >= 1/2}, and per-drop volumes matched
    by root (the drop's smallest cell index)."""
    import numpy as np
    (r32, c32), (r64, c64) = drops32, drops64
    v32 = float(np.sum(c32)) * h ** 3
    v64 = float(np.sum(c64)) * h ** 3
    by64 = dict(zip(r64.tolist(), c64.tolist()))
    matched = [(c, by64[r]) for r, c in zip(r32.tolist(), c32.tolist()) if r in by64]
    return {"steps": steps,
            "l2_rel": float(np.linalg.norm(C32 - C64) / np.linalg.norm(C64)),
            "mass_drift_fp32": abs(m32[1] - m32[0]) / abs(m32[0]),
            "mass_drift_fp64": abs(m64[1] - m64[0]) / abs(m64[0]),
            "drop_volume_err": abs(v32 - v64) / v64 if v64 > 0 else None,
            "drops": {"definition": DROPS_DEF, "count_fp32": int(len(r32)),
                      "count_fp64": int(len(r64)), "matched_by_root": len(matched),
                      "max_rel_volume_err_fp32_vs_fp64":
                          max((abs(a - b) / b for a, b in matched), default=None),
                      "l_loss_fp32": (m32[1] - m32[0]) / m32[0],
                      "l_loss_fp64": (m64[1] - m64[0]) / m64[0],
                      "D_over_H_pdf_fp64": dh_histogram(c64, h, H)}}


def counter_probe(prec="fp32"):
    """A short run for rocprofv3 counter passes: two steps of the workload
    (FP32 unless `prec` says otherwise), then one device-to-device copy of
    256 MiB (the kernel whose FETCH_SIZE / WRITE_SIZE readings calibrate the
    counters)."""
    import torch
    from paper_2105_01865_amd import ch, inputs
    stream = torch.cuda.Stream()
    if prec == "large":
        # one step of the 1536^3 box, in the bench's automatic plan
        from paper_2105_01865_amd import inputs_gpu
        wl = inputs_gpu.large_workload()
        s = ch.State(wl.shape, wl.h, wl.Cn, wl.Pe, precision="fp32", stream=stream)
        s.set_field(wl.C)
        del wl.C
        torch.cuda.empty_cache()
        s.step(wl.u, wl.v, wl.w, wl.dt, 1)
        torch.cuda.synchronize()
        s.close()
        del wl
        torch.cuda.empty_cache()
    else:
        wl = inputs.make_workload(2)
        dt_ = torch.float64 if prec == "fp64" else torch.float32
        s = ch.State(wl.shape, wl.h, wl.Cn, wl.Pe, precision=prec, stream=stream)
        s.set_field(torch.from_numpy(wl.C).to("cuda", dt_))
        U, V, W = (torch.from_numpy(a).to("cuda", dt_) for a in (wl.u, wl.v, wl.w))
        s.step(U, V, W, wl.dt, 2)
        torch.cuda.synchronize()
        s.close()
    a = torch.ones(64 << 20, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print("counter probe done", flush=True)


def _timed_events(stream, fn):
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def bench_ensemble(args, stream):
    """The batched ensemble: 48 independent periodic boxes with edges from
    {48, 64, 96, 128, 160, 192}, 1-20 drops each, per-box ABC flows; all boxes
    advance in one graph launch per step.  Each precision steps from the
    same initial fields: warm-up, the timed steps, then on to --acc-steps
    steps in all, for the FP32-vs-FP64 errors."""
    import numpy as np
    from paper_2105_01865_amd import ch, inputs
    E = inputs.ensemble(48)
    pts = sum(w.points for w in E)
    res = {}
    fields = {}
    drops = {}
    masses = {}
    nacc = 0
    for prec in ("fp32", "fp64"):
        b = ch.Batch([w.shape for w in E], [w.h for w in E], [w.Cn for w in E],
                     [w.Pe for w in E], stream=stream, precision=prec)
        U, V, W = (b.pack([getattr(w, f) for w in E], f) for f in "uvw")
        b.set_field(b.pack([w.C for w in E], "c"))
        tune = b.autotune(U, V, W, 1e-4, steps=5) if not args.no_autotune else None
        m0 = np.array(b.mass())
        b.step(U, V, W, 1e-4, args.warmup)
        ms = _timed_events(stream, lambda: b.step(U, V, W, 1e-4, args.ensemble_steps))
        done = args.warmup + args.ensemble_steps
        if args.acc_steps > done:
            b.step(U, V, W, 1e-4, args.acc_steps - done)
        nacc = max(done, args.acc_steps)
        m1 = np.array(b.mass())
        masses[prec] = (m0, m1)
        fields[prec] = b.unpack(b.get_field())
        fields[prec] = [f.double().cpu().numpy() for f in fields[prec]]
        drops[prec] = [b.drops(i) for i in range(len(E))]
        b.profile(True)
        b.step(U, V, W, 1e-4, 5)
        kern = {k: b.profile_read(k) for k in ("x", "y", "z")}
        b.profile(False)
        b.close()
        es = 4 if prec == "fp32" else 8
        x_us = 1e3 * kern["x"][0] / max(1, kern["x"][1])
        res[prec] = {"value": round(pts * args.ensemble_steps / (ms * 1e-3) / 1e9, 4),
                     "unit": "Gpts/s", "ms_per_step": round(ms / args.ensemble_steps, 4),
                     "max_box_mass_drift": float(np.max(np.abs(m1 - m0) / np.abs(m0))),
                     "autotune": tune,
                     "kernels_avg_us": {k: round(1e3 * v[0] / max(1, v[1]), 1)
                                        for k, v in kern.items()},
                     "hbm_frac_step_model": step_hbm_frac(pts, es, ms / args.ensemble_steps),
                     "roofline": x_roofline(x_us, pts, es)}
    # FP32 against FP64, box by box
    l2n = sum(float(np.sum((a - c) ** 2)) for a, c in zip(fields["fp32"], fields["fp64"]))
    l2d = sum(float(np.sum(c ** 2)) for c in fields["fp64"])
    vol_err, drop_err, cnt = [], [], [0, 0]
    for i, w in enumerate(E):
        (r32, c32), (r64, c64) = drops["fp32"][i], drops["fp64"][i]
        cnt[0] += len(r32)
        cnt[1] += len(r64)
        v64 = float(np.sum(c64))
        if v64 > 0:
            vol_err.append(abs(float(np.sum(c32)) - v64) / v64)
        by64 = dict(zip(r64.tolist(), c64.tolist()))
        drop_err += [abs(c - by64[r]) / by64[r] for r, c in zip(r32.tolist(), c32.tolist())
                     if r in by64]
    (a0, a1), (b0, b1) = masses["fp32"], masses["fp64"]
    acc = {"steps": nacc, "l2_rel": (l2n / l2d) ** 0.5,
           "max_box_mass_drift_fp32": float(np.max(np.abs(a1 - a0) / np.abs(a0))),
           "max_box_mass_drift_fp64": float(np.max(np.abs(b1 - b0) / np.abs(b0))),
           "max_box_drop_volume_err": max(vol_err) if vol_err else None,
           "drops": {"definition": DROPS_DEF, "count_fp32": cnt[0], "count_fp64": cnt[1],
                     "matched_by_root": len(drop_err),
                     "max_rel_volume_err_fp32_vs_fp64": max(drop_err) if drop_err else None}}
    return {"workload": "48 periodic boxes, edge ~ U{48,64,96,128,160,192}, h = 1/edge, "
                        "1-20 tanh drops R~U[4,12]h, ABC flow A,B,C~U[0.05,0.2], dt=1e-4",
            "points": pts, "steps": args.ensemble_steps, "fp32": res["fp32"], "fp64": res["fp64"],
            "fp32_over_fp64": round(res["fp32"]["value"] / res["fp64"]["value"], 3),
            "accuracy_fp32_vs_fp64": acc, "roofline": res["fp32"]["roofline"]}


def transfer_bytes_per_component(nc, nf, es):
    """Algorithmic HBM bytes of one component of the plain coarse-to-fine
    transfer: every coarse value read once, every fine value written once."""
    ncz, ncy, ncx = nc
    nz, ny, nx = nf
    return (ncx * ncy * ncz + nx * ny * nz) * es


def bench_multires(args, stream):
    """The multiple-resolution workload: 512^3 fine mesh, periodic in x and y,
    no-flux walls in z, 1000 drops; the velocity lives on a 256 x 256 x 192
    mesh stretched in z and is transferred to the fine faces every step,
    by the plain transfer and by the solenoidal one."""
    import numpy as np
    import torch
    from paper_2105_01865_amd import ch, inputs
    wl = inputs.make_workload(3)
    zf, uc, vc, wc = (wl.coarse[k] for k in ("zf", "uc", "vc", "wc"))
    res = {}
    fields = {}
    masses = {}
    drops = {}
    nacc = 0
    for prec in ("fp32", "fp64"):
        dt_ = torch.float32 if prec == "fp32" else torch.float64
        es = 4 if prec == "fp32" else 8
        UC, VC, WC = (torch.from_numpy(a).to("cuda", dt_) for a in (uc, vc, wc))
        C0 = torch.from_numpy(wl.C).to("cuda", dt_)
        for mode in ("plain", "solenoidal"):
            s = ch.State(wl.shape, wl.h, wl.Cn, wl.Pe, bc=wl.bc, precision=prec, stream=stream)
            ip = ch.Interp(wl.shape, wl.h, uc.shape, zf, precision=prec, stream=stream,
                           solenoidal=mode == "solenoidal")
            s.set_field(C0)
            tune = None
            if not args.no_autotune:
                # the step's tiles, tuned on the transferred velocity
                tune = s.autotune(*ip.apply(UC, VC, WC), wl.dt, steps=3)
            m0 = s.mass()
            s.step_multires(ip, UC, VC, WC, wl.dt, args.warmup)
            ms = _timed_events(stream, lambda: s.step_multires(ip, UC, VC, WC, wl.dt,
                                                               args.multires_steps))
            if mode == "plain":
                # on to --multires-acc-steps steps from the initial field
                done = args.warmup + args.multires_steps
                if args.multires_acc_steps > done:
                    s.step_multires(ip, UC, VC, WC, wl.dt, args.multires_acc_steps - done)
                nacc = max(done, args.multires_acc_steps)
            m1 = s.mass()
            if mode == "plain":
                fields[prec] = s.get_field().double().cpu().numpy()
                masses[prec] = (m0, m1)
                drops[prec] = s.drops()
            s.profile(True)
            s.step_multires(ip, UC, VC, WC, wl.dt, 5)
            kern = {k: s.profile_read(k) for k in ("x", "y", "z", "interp")}
            s.profile(False)
            clo = ip.closure()
            s.close()
            ip.close()
            t_us = 1e3 * kern["interp"][0] / max(1, kern["interp"][1])
            x_us = 1e3 * kern["x"][0] / max(1, kern["x"][1])
            nbytes = transfer_bytes_per_component(uc.shape, wl.shape, es)
            r = {"value": round(wl.points * args.multires_steps / (ms * 1e-3) / 1e9, 4),
                 "unit": "Gpts/s", "ms_per_step": round(ms / args.multires_steps, 4),
                 "mass_drift": abs(m1 - m0) / abs(m0), "autotune": tune,
                 "kernels_avg_us": {k: round(1e3 * v[0] / max(1, v[1]), 1)
                                    for k, v in kern.items()},
                 "roofline": x_roofline(x_us, wl.points, es)}
            if mode == "plain":
                # the step's 34 element accesses per point plus three transfers
                r["hbm_frac_step_model"] = step_hbm_frac(wl.points, es, ms / args.multires_steps,
                                                         3 * nbytes)
            if mode == "plain":
                # the transfer of one component is one k_interp launch
                r["transfer_roofline"] = {
                    "bound": "hbm", "bytes_per_component": nbytes,
                    "achieved_GBs": round(nbytes / (t_us * 1e-6) / 1e9, 1),
                    "peak_GBs": HBM_PEAK_GBS,
                    "frac": round(nbytes / (t_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 3)}
            else:
                # gradient, interpolation to the fine centres, reference plane
                # and in-place integration: the fine array is written, read
                # and written again
                sb = nbytes + 2 * (wl.points * es) + 2 * (uc.size * es)
                r["transfer_roofline"] = {
                    "bound": "hbm", "bytes_per_component": sb,
                    "achieved_GBs": round(sb / (t_us * 1e-6) / 1e9, 1),
                    "peak_GBs": HBM_PEAK_GBS,
                    "frac": round(sb / (t_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 3),
                    "vs_plain_transfer_bytes": round(sb / nbytes, 2)}
                r["closure_max"] = [float(c) for c in clo]
            res.setdefault(prec, {})[mode] = r
        del UC, VC, WC, C0
    acc = fp32_errors(fields["fp32"], fields["fp64"], masses["fp32"], masses["fp64"],
                      drops["fp32"], drops["fp64"], wl.h, wl.shape[0] * wl.h, nacc)
    return {"workload": "512^3 fine mesh, periodic x,y, no-flux z, 1000 tanh drops R~U[4,12]h; "
                        "velocity on 256x256x192 (tanh-stretched z) transferred every step "
                        "(transfer inside the step time), plain and solenoidal transfer",
            "points": wl.points, "steps": args.multires_steps, "dt": wl.dt,
            "fp32": res["fp32"]["plain"], "fp64": res["fp64"]["plain"],
            "solenoidal": {"fp32": res["fp32"]["solenoidal"], "fp64": res["fp64"]["solenoidal"]},
            "fp32_over_fp64": round(res["fp32"]["plain"]["value"] / res["fp64"]["plain"]["value"], 3),
            "accuracy_fp32_vs_fp64": acc, "roofline": res["fp32"]["plain"]["roofline"]}


def pressure_bytes_per_step(n, es):
    """Algorithmic HBM bytes of one pressure step on n cells: element accesses
    prep 4 (P, Pold in; Phat, Pold out), right-hand side 6 (C, Phat, u, v, w
    in; rhs out), forward transform 2, mode solves 3 (spectrum in and out,
    half a field of Thomas scratch written and read), inverse transform 2,
    update 9 (C, P, Phat, u, v, w in; u, v, w out): 26 n elements."""
    return 26 * n * es


def bench_pressure(args, stream):
    """The split-density pressure step on the 512^3 multiple-resolution box
    (walls in z): C and u* from that workload (u* = the plain transfer of
    its coarse velocity), density ratio 1000, P and P^{l-1} from the steps
    before."""
    import torch
    from paper_2105_01865_amd import ch, inputs
    wl = inputs.make_workload(3)
    zf, uc, vc, wc = (wl.coarse[k] for k in ("zf", "uc", "vc", "wc"))
    res = {}
    for prec in ("fp32", "fp64"):
        dt_ = torch.float32 if prec == "fp32" else torch.float64
        es = 4 if prec == "fp32" else 8
        ip = ch.Interp(wl.shape, wl.h, uc.shape, zf, precision=prec, stream=stream)
        u0, v0, w0 = ip.apply(*(torch.from_numpy(a).to("cuda", dt_) for a in (uc, vc, wc)))
        ip.close()
        C = torch.from_numpy(wl.C).to("cuda", dt_)
        P = torch.zeros(wl.shape, dtype=dt_, device="cuda")
        Pold = torch.zeros_like(P)
        p = ch.Poisson(wl.shape, wl.h, z_walls=True, precision=prec, stream=stream)
        u, v, w = u0.clone(), v0.clone(), w0.clone()
        for _ in range(args.warmup):
            u.copy_(u0), v.copy_(v0), w.copy_(w0)
            p.step(C, u, v, w, P, Pold, 1000.0, 1.0, wl.dt)
        torch.cuda.synchronize()
        n = args.pressure_steps
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * n)]
        for k in range(n):
            u.copy_(u0), v.copy_(v0), w.copy_(w0)
            ev[2 * k].record(stream)
            p.step(C, u, v, w, P, Pold, 1000.0, 1.0, wl.dt)
            ev[2 * k + 1].record(stream)
        torch.cuda.synchronize()
        ms = sum(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(n)) / n
        h = wl.h
        div = ((torch.roll(u, -1, 2) - u) + (torch.roll(v, -1, 1) - v) + (w[1:] - w[:-1])) / h
        div0 = ((torch.roll(u0, -1, 2) - u0) + (torch.roll(v0, -1, 1) - v0) + (w0[1:] - w0[:-1])) / h
        nbytes = pressure_bytes_per_step(wl.points, es)
        res[prec] = {"ms_per_step": round(ms, 4),
                     "Gpts_per_s": round(wl.points / (ms * 1e-3) / 1e9, 3),
                     "max_div_after_over_before": float(div.abs().max() / div0.abs().max()),
                     "roofline": {"bound": "hbm", "bytes_per_step": nbytes,
                                  "achieved_GBs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                                  "peak_GBs": HBM_PEAK_GBS,
                                  "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)}}
        p.close()
        del u, v, w, u0, v0, w0, C, P, Pold
    return {"workload": "512^3 cells, periodic x,y, walls in z; C of the 1000-drop workload, "
                        "u* its transferred velocity, rho1/rho2 = 1000, dt = 1e-4",
            "points": wl.points, "steps": args.pressure_steps,
            "fp32": res["fp32"], "fp64": res["fp64"]}


def bench_large(args, stream):
    """The 1536^3 periodic box in single precision (inputs built on the GPU):
    FP32 throughput over a few steps, and the whole box's mass drift."""
    import torch
    from paper_2105_01865_amd import ch, inputs_gpu
    torch.cuda.empty_cache()
    wl = inputs_gpu.large_workload()
    s = ch.State(wl.shape, wl.h, wl.Cn, wl.Pe, precision="fp32", stream=stream)
    s.set_field(wl.C)
    del wl.C
    tune = s.autotune(wl.u, wl.v, wl.w, wl.dt, steps=2) if not args.no_autotune else None
    m0 = s.mass()
    s.step(wl.u, wl.v, wl.w, wl.dt, 1)
    ms = _timed_events(stream, lambda: s.step(wl.u, wl.v, wl.w, wl.dt, args.large_steps))
    m1 = s.mass()
    s.profile(True)
    s.step(wl.u, wl.v, wl.w, wl.dt, 2)
    kern = {k: s.profile_read(k) for k in ("x", "y", "z")}
    s.profile(False)
    cfg = s.config()
    s.close()
    dt = wl.dt
    del wl
    torch.cuda.empty_cache()
    pts = 1536 ** 3
    x_us = 1e3 * kern["x"][0] / max(1, kern["x"][1])
    return {"workload": "1536^3 periodic box, FP32 storage, 4000 tanh drops R~U[4,20]h, "
                        "k^-5/3 field 1<=k<=48 rms 1 (inputs generated on the GPU), "
                        "dt from the advective bound",
            "points": pts, "steps": args.large_steps, "dt": dt,
            "fp32": {"value": round(pts * args.large_steps / (ms * 1e-3) / 1e9, 4),
                     "unit": "Gpts/s", "ms_per_step": round(ms / args.large_steps, 3),
                     "mass_drift": abs(m1 - m0) / abs(m0),
                     "kernels_avg_us": {k: round(1e3 * v[0] / max(1, v[1]), 1)
                                        for k, v in kern.items()},
                     "hbm_frac_step_model": step_hbm_frac(pts, 4, ms / args.large_steps)},
            "roofline": dict(x_roofline(x_us, pts, 4, measured_traffic(TRAFFIC_FILE_LARGE)),
                             issue_view=issue_view(x_us, SQ_FILE_LARGE),
                             limit=limiter(issue_view(x_us, SQ_FILE_LARGE),
                                           measured_traffic(TRAFFIC_FILE_LARGE), x_us)),
            "plan": cfg, "autotune": tune}


def bench_subbox(args, stream, dt):
    """The error reference of the 1536^3 workload: its 256^3 sub-box (same h,
    the drops inside it, the velocity modes periodic on it) run in FP32 and
    FP64 for --subbox-steps steps with the 1536^3 run's dt."""
    import torch
    from paper_2105_01865_amd import ch, inputs
    wl = inputs.large_subbox()
    out = {}
    for prec in ("fp32", "fp64"):
        dt_ = torch.float32 if prec == "fp32" else torch.float64
        s = ch.State(wl.shape, wl.h, wl.Cn, wl.Pe, precision=prec, stream=stream)
        s.set_field(torch.from_numpy(wl.C).to("cuda", dt_))
        U, V, W = (torch.from_numpy(a).to("cuda", dt_) for a in (wl.u, wl.v, wl.w))
        m0 = s.mass()
        s.step(U, V, W, dt, args.subbox_steps)
        m1 = s.mass()
        out[prec] = (s.get_field().double().cpu().numpy(), (m0, m1), s.drops())
        s.close()
    acc = fp32_errors(out["fp32"][0], out["fp64"][0], out["fp32"][1], out["fp64"][1],
                      out["fp32"][2], out["fp64"][2], wl.h, wl.shape[0] * wl.h,
                      args.subbox_steps)
    return {"workload": "256^3 sub-box of the 1536^3 workload: h = 1/1536, the "
                        f"{wl.ndrops} drops lying inside it, k^-5/3 modes periodic on it "
                        "(big-box k = 6..48) at their share of the rms",
            "dt": dt, **acc}


def bench_host_io(args, stream, wl, tune):
    """The 256^3 FP32 box with C handed over in host memory: C copied in from
    pinned host memory through ch_set_field, `steps_per_trip` steps, C copied
    back out through ch_get_field, the velocity resident on the GPU.  Host
    wall time of whole round trips (the copies wait for the stream)."""
    import numpy as np
    import torch
    from paper_2105_01865_amd import ch
    pts = wl.points
    U, V, W = (torch.from_numpy(a).to(device="cuda", dtype=torch.float32)
               for a in (wl.u, wl.v, wl.w))
    hC = torch.from_numpy(wl.C.astype(np.float32)).pin_memory()
    out = torch.empty(wl.shape, dtype=torch.float32).pin_memory()
    plan = ({k: tune[k] for k in ("x_rows", "z_chunk", "seg_len")} if tune else {})
    s = ch.State(wl.shape, wl.h, wl.Cn, wl.Pe, precision="fp32", stream=stream, **plan)
    s.set_field_host(hC)
    s.step(U, V, W, wl.dt, 2)
    s.get_field_host(out)
    res = {}
    for k in (1, 10):
        t_in, t_step, t_out = [], [], []
        for _ in range(args.host_io_reps):
            t0 = time.perf_counter()
            s.set_field_host(hC)
            t1 = time.perf_counter()
            s.step(U, V, W, wl.dt, k)
            stream.synchronize()
            t2 = time.perf_counter()
            s.get_field_host(out)
            t3 = time.perf_counter()
            t_in.append(t1 - t0)
            t_step.append(t2 - t1)
            t_out.append(t3 - t2)
        med = lambda a: float(np.median(a))
        trip = med([a + b + c for a, b, c in zip(t_in, t_step, t_out)])
        res[f"steps_per_trip_{k}"] = {"value": round(pts * k / trip / 1e9, 4), "unit": "Gpts/s",
                                      "trip_ms": round(trip * 1e3, 3),
                                      "h2d_ms": round(med(t_in) * 1e3, 3),
                                      "steps_ms": round(med(t_step) * 1e3, 3),
                                      "d2h_ms": round(med(t_out) * 1e3, 3)}
    s.close()
    nbytes = pts * 4
    r1 = res["steps_per_trip_1"]
    return {"workload": "256^3 FP32 box, C in and out through pinned host memory each trip, "
                        "velocity resident, the headline's launch plan",
            "reps": args.host_io_reps, "field_bytes": nbytes,
            "h2d_gbs": round(nbytes / (r1["h2d_ms"] * 1e-3) / 1e9, 1),
            "d2h_gbs": round(nbytes / (r1["d2h_ms"] * 1e-3) / 1e9, 1), **res}


def bench_explicit25(args, stream, line):
    """The paper's starting point, the explicit 25-point biharmonic (no line
    solves), on the same 256^3 workload: its throughput at 0.85 of the
    biharmonic's RK3 stability bound (advection and the psi'' term move the
    practical limit to 0.90-0.95 of it at 256^3), stability checked at 0.85
    and 1.05 of the bound, and the time to reach a given simulated time
    against the implicit scheme at the workload's dt."""
    import numpy as np
    import torch
    from paper_2105_01865_amd import ch, inputs
    wl = inputs.make_workload(2)
    # highest mode of the 25-point operator: 144 Cn^2/h^4; RK3 real-axis bound
    zmax = 2.5127453266183286
    dt_lim = zmax * wl.Pe / (144.0 * wl.Cn ** 2 / wl.h ** 4)
    res = {}
    for prec in ("fp32", "fp64"):
        dt_ = torch.float32 if prec == "fp32" else torch.float64
        U, V, W = (torch.from_numpy(a).to("cuda", dt_) for a in (wl.u, wl.v, wl.w))
        C0 = torch.from_numpy(wl.C).to("cuda", dt_)
        s = ch.State(wl.shape, wl.h, wl.Cn, wl.Pe, precision=prec, stream=stream)
        s.set_field(C0)
        s.step_explicit25(U, V, W, 0.85 * dt_lim, args.warmup)
        ms = _timed_events(stream, lambda: s.step_explicit25(U, V, W, 0.85 * dt_lim,
                                                             args.explicit_steps))
        res[prec] = {"value": round(wl.points * args.explicit_steps / (ms * 1e-3) / 1e9, 4),
                     "unit": "Gpts/s", "ms_per_step": round(ms / args.explicit_steps, 4)}
        if prec == "fp32":
            growth = {}
            for f in (0.85, 1.05):
                s.set_field(C0)
                s.step_explicit25(U, V, W, f * dt_lim, args.explicit_steps)
                C = s.get_field().double().cpu().numpy()
                growth[str(f)] = float(np.abs(C - 0.5).max()) if np.all(np.isfinite(C)) else None
            res["max_abs_C_minus_half_after_steps"] = growth
        s.close()
    impl32 = line["ms_per_step"]
    impl_dt = wl.dt
    tts = (res["fp32"]["ms_per_step"] / (0.85 * dt_lim)) / (impl32 / impl_dt)
    return {"workload": line["config"]["workload"] + "; explicit 25-point biharmonic",
            "dt_bound_biharmonic": dt_lim, "dt_used": 0.85 * dt_lim,
            "steps": args.explicit_steps,
            "fp32": res["fp32"], "fp64": res["fp64"],
            "stability_check_fp32": res["max_abs_C_minus_half_after_steps"],
            "implicit_dt": impl_dt,
            "time_to_solution_explicit_over_implicit_fp32": round(tts, 3)}


def _oracle_rate(step_fn, points_per_step, tmin, tmax):
    """Whole oracle steps until tmin seconds of work (at least one step,
    stopping before tmax): (Gpts/s, steps, seconds)."""
    steps = 0
    t0 = time.perf_counter()
    while True:
        step_fn()
        steps += 1
        el = time.perf_counter() - t0
        if el >= tmin or el / steps * (steps + 1) > tmax:
            break
    return points_per_step * steps / el / 1e9, steps, el


def cpu_baselines(wl, args):
    """The FP64 oracle timed on this host: the 256^3 workload on all cores
    (whole steps until about 10 s, the line's cpu_baseline figure) and on one
    core (one step), then bounded samples of the other workloads: the 32^3
    box on all cores and on one, the multiple-resolution recipe shrunk to
    256^3 (transfer + step), one box of each edge of the ensemble, and the
    1536^3 workload's 256^3 sub-box."""
    import oracle
    from paper_2105_01865_amd import inputs
    cores = oracle.threads()
    C = [wl.C]

    def step_of(w, bc=(0, 0, 0), dt=None):
        def f():
            C[0] = oracle.step(C[0], w.u, w.v, w.w, w.h, w.Cn, w.Pe, dt or w.dt, 1, bc=bc)
        return f

    v, n, el = _oracle_rate(step_of(wl), wl.points, 10.0, 30.0)
    out = {"value": round(v, 6), "unit": "Gpts/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} RK3 step(s) of the same {wl.shape[2]}^3 workload in FP64, "
                     f"{el:.1f} s, on all {cores} threads"}
    others = {}
    try:
        oracle.set_threads(1)
        C[0] = wl.C
        v, n, el = _oracle_rate(step_of(wl), wl.points, 0.0, 1e9)
        out["one_core"] = {"value": round(v, 6), "unit": "Gpts/s", "cores": 1,
                           "sample": f"{n} step of the {wl.shape[2]}^3 workload, {el:.1f} s"}
        w1 = inputs.make_workload(1)
        C[0] = w1.C
        v, n, el = _oracle_rate(step_of(w1), w1.points, 2.0, 10.0)
        others["32cube_one_core"] = {"value": round(v, 6), "cores": 1,
                                     "sample": f"{n} steps, {el:.1f} s"}
    finally:
        oracle.set_threads(cores)
    C[0] = w1.C
    v, n, el = _oracle_rate(step_of(w1), w1.points, 2.0, 10.0)
    others["32cube"] = {"value": round(v, 6), "cores": cores, "sample": f"{n} steps, {el:.1f} s"}
    # the multiple-resolution recipe at 256^3: transfer from the coarse mesh
    # and step, every step
    w3 = inputs.make_workload(3, n=256)
    zf, uc, vc, wc = (w3.coarse[k] for k in ("zf", "uc", "vc", "wc"))
    C[0] = w3.C

    def step3():
        u, v_, w_ = oracle.interp_velocity(zf, uc, vc, wc, w3.shape)
        C[0] = oracle.step(C[0], u, v_, w_, w3.h, w3.Cn, w3.Pe, w3.dt, 1, bc=(0, 0, 1))

    v, n, el = _oracle_rate(step3, w3.points, 2.0, 30.0)
    others["multires_recipe_256cube"] = {"value": round(v, 6), "cores": cores,
                                         "sample": f"{n} steps (transfer + step), {el:.1f} s"}
    # one box of each ensemble edge, one step each
    E = inputs.ensemble(48)
    picks = [next(w for w in E if w.shape[0] == e) for e in (48, 64, 96, 128, 160, 192)]
    t0 = time.perf_counter()
    for w in picks:
        oracle.step(w.C, w.u, w.v, w.w, w.h, w.Cn, w.Pe, w.dt, 1)
    el = time.perf_counter() - t0
    others["ensemble_one_box_per_edge"] = {
        "value": round(sum(w.points for w in picks) / el / 1e9, 6), "cores": cores,
        "sample": f"one step of one box of each edge 48..192, {el:.1f} s"}
    sb = inputs.large_subbox()
    C[0] = sb.C
    v, n, el = _oracle_rate(step_of(sb, dt=4e-5), sb.points, 1.0, 30.0)
    others["large_subbox_256cube"] = {"value": round(v, 6), "cores": cores,
                                      "sample": f"{n} step(s), {el:.1f} s"}
    out["other_workloads"] = others
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=200)
    ap.add_argument("--multires-steps", type=int, default=100)
    ap.add_argument("--large-steps", type=int, default=10)
    ap.add_argument("--explicit-steps", type=int, default=200)
    ap.add_argument("--pressure-steps", type=int, default=20)
    ap.add_argument("--host-io-reps", type=int, default=20)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the planner's automatic tiles (no launch-plan autotuning)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched-ensemble and multiple-resolution lines")
    ap.add_argument("--counter-probe", nargs="?", const="fp32", default=None,
                    choices=("fp32", "fp64", "large"),
                    help="two steps of the 256^3 box (or one of the 1536^3 box) and a "
                         "256 MiB copy, for rocprofv3 counter runs")
    ap.add_argument("--acc-steps", type=int, default=1000,
                    help="steps of the FP32-vs-FP64 accuracy leg of the 256^3 box and the "
                         "ensemble (independent of --steps)")
    ap.add_argument("--multires-acc-steps", type=int, default=500,
                    help="steps of the multiple-resolution accuracy leg")
    ap.add_argument("--subbox-steps", type=int, default=200,
                    help="steps of the 1536^3 workload's 256^3 sub-box error reference")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library "
              "has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.counter_probe:
        counter_probe(args.counter_probe)
        return

    import numpy as np
    import torch

    from paper_2105_01865_amd import ch, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = inputs.make_workload(2)
    pts = wl.points
    stream = torch.cuda.Stream()
    h = wl.h

    def timed(prec):
        dt_ = torch.float64 if prec == "fp64" else torch.float32
        s = ch.State(wl.shape, h, wl.Cn, wl.Pe, precision=prec, stream=stream)
        C0 = torch.from_numpy(wl.C).to(device="cuda", dtype=dt_)
        U, V, W = (torch.from_numpy(a).to(device="cuda", dtype=dt_) for a in (wl.u, wl.v, wl.w))
        s.set_field(C0)
        # launch-plan autotuning (before the timed region; C is restored)
        tune = s.autotune(U, V, W, wl.dt, steps=10) if not args.no_autotune else None
        m0 = s.mass()
        s.step(U, V, W, wl.dt, args.warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        s.step(U, V, W, wl.dt, args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        # on to --acc-steps steps from the initial field (accuracy leg)
        done = args.warmup + args.steps
        if args.acc_steps > done:
            s.step(U, V, W, wl.dt, args.acc_steps - done)
        m1 = s.mass()
        C = s.get_field().double().cpu().numpy()
        cfg = s.config()
        # drops of the final field (the first call allocates the labels)
        s.drops()
        t0 = time.perf_counter()
        roots, cells = s.drops()
        label_ms = (time.perf_counter() - t0) * 1e3
        # every kernel, timed launch by launch with HIP events on the
        # library's stream over a profiled run of the same steps
        s.set_field(C0)
        s.profile(True)
        s.step(U, V, W, wl.dt, args.profile_steps)
        prof = {k: s.profile_read(k) for k in ("x", "y", "z")}
        s.profile(False)
        s.close()
        return dict(ms=ms, wall=wall, m0=m0, m1=m1, C=C, cfg=cfg, prof=prof, roots=roots,
                    cells=cells, label_ms=label_ms, tune=tune, nacc=max(done, args.acc_steps))

    r32 = timed("fp32")
    progress("256^3 fp32 done")
    r64 = timed("fp64")
    progress("256^3 fp64 done")
    nstep = args.steps
    v32 = pts * nstep / (r32["ms"] * 1e-3) / 1e9
    v64 = pts * nstep / (r64["ms"] * 1e-3) / 1e9

    # accuracy of FP32 against FP64 after --acc-steps steps from the same field
    acc = fp32_errors(r32["C"], r64["C"], (r32["m0"], r32["m1"]), (r64["m0"], r64["m1"]),
                      (r32["roots"], r32["cells"]), (r64["roots"], r64["cells"]), h,
                      wl.shape[0] * h, r32["nacc"])
    acc["drops"]["label_ms_fp32"] = round(r32["label_ms"], 2)
    acc["drops"]["label_ms_fp64"] = round(r64["label_ms"], 2)
    acc["drops"]["label_ms_note"] = "ch_drops wall time: labelling, counting, copy-out and sort"

    def kern(r):
        return {k: dict(avg_us=round(1e3 * r["prof"][k][0] / max(1, r["prof"][k][1]), 2),
                        launches=r["prof"][k][1]) for k in ("x", "y", "z")}

    # roofline of the x pass (FP32 run: the headline precision)
    xms, xn = r32["prof"]["x"]
    x_avg_s = xms / xn * 1e-3
    x_flops = x_pass_flops_per_point() * pts
    achieved = x_flops / x_avg_s / 1e12
    traffic = measured_traffic()
    roof = x_roofline(x_avg_s * 1e6, pts, 4, traffic,
                      kernel="k_pass_x (explicit terms + RHS + x solve), fp32")
    roof.update({
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                        "copy-calibrated)",
        "bytes_per_point": x_pass_bytes_per_point(4),
        "measured_gbs": round(traffic / x_avg_s / 1e9, 1) if traffic else None,
        "measured_frac": round(traffic / x_avg_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
        "traffic_over_algorithmic": (round(traffic / roof["algorithmic_bytes_per_launch"], 3)
                                     if traffic else None),
        # the same launch against the vector ALUs (the pass issues more VALU
        # instructions than its algorithmic flops)
        "alu_view": {"flops_per_point": x_pass_flops_per_point(),
                     "achieved_tflops": round(achieved, 3),
                     "peak_published_fp32_tflops": VALU_PEAK_PUBLISHED_FP32_TFLOPS,
                     "frac_published": round(achieved / VALU_PEAK_PUBLISHED_FP32_TFLOPS, 4),
                     "peak_nonpacked_tflops": VALU_PEAK_TFLOPS,
                     "frac_nonpacked": round(achieved / VALU_PEAK_TFLOPS, 4)},
        # and against vector instruction issue, the limit it runs at
        "issue_view": issue_view(x_avg_s * 1e6),
        "limit": limiter(issue_view(x_avg_s * 1e6), traffic, x_avg_s * 1e6),
        "window": f"{args.profile_steps} profiled steps, HIP events per launch"})

    line = {
        "metric": METRIC,
        "value": round(v32, 4),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": nstep,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms"] / nstep, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded drops + k^-5/3 divergence-free field)",
        "config": {"workload": f"{wl.shape[2]}^3 periodic CH box, {wl.ndrops} tanh drops "
                               "R~U[6,16]h, frozen k^-5/3 field 1<=k<=16 rms 1, Cn=h, "
                               "Pe=0.9/Cn, dt=1e-4, kappa=4",
                   "points": pts, "precision": "fp32 storage+stencils, fp64 mass",
                   "plan": r32["cfg"], "autotune": r32["tune"]},
        "fp64": {"value": round(v64, 4), "unit": "Gpts/s",
                 "ms_per_step": round(r64["ms"] / nstep, 5), "plan": r64["cfg"],
                 "autotune": r64["tune"]},
        "fp32_over_fp64": round(v32 / v64, 3),
        "accuracy_fp32_vs_fp64": acc,
        "hbm_frac_step_model": step_hbm_frac(pts, 4, r32["ms"] / nstep),
        "hbm_frac_step_model_fp64": step_hbm_frac(pts, 8, r64["ms"] / nstep),
        "roofline": roof,
        "kernels_fp32": kern(r32),
        "kernels_fp64": kern(r64),
    }

    line["host_io"] = bench_host_io(args, stream, wl, r32["tune"])
    progress("host-memory round trips done")
    if not args.no_extra:
        line["batched"] = bench_ensemble(args, stream)
        progress("ensemble done")
        line["multires"] = bench_multires(args, stream)
        progress("multiple resolution done")
        line["pressure"] = bench_pressure(args, stream)
        progress("pressure step done")
        line["large"] = bench_large(args, stream)
        progress("1536^3 done")
        line["large"]["subbox_accuracy_fp32_vs_fp64"] = bench_subbox(args, stream,
                                                                     line["large"]["dt"])
        progress("1536^3 sub-box accuracy done")
        line["explicit25"] = bench_explicit25(args, stream, line)
        progress("explicit 25-point done")

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baselines(wl, args)
        progress("cpu baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
