"""Benchmark of the Cahn-Hilliard update on one MI355X.

Workload: the 256^3 periodic box with 64 tanh drops (radii 6-16 h) in a
frozen divergence-free k^-5/3 velocity field (1 <= k <= 16, rms 1),
Cn = h, Pe = 0.9/Cn, dt = 1e-4.  Inputs are seeded and synthetic and are
resident in HBM before the timed region starts.

A step is one full RK3 step (3 substages x {x pass, y solve, z solve}).
`value` is the FP32 throughput in grid-point updates per second (Gpts/s);
the FP64 throughput, the FP32-vs-FP64 error after warmup + timed steps, the
roofline of the dominant kernel (the x pass) and the FP64 CPU oracle's
throughput on a bounded sample of the same workload are reported on the
same JSON line.

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
METRIC = ("CH grid-point updates/s (Gpts/s) FP32 & batched vs FP64 at stated error; "
          "%HBM peak")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pass_x_256cube_fp32_traffic.md")
X_SOURCES = ("ch_device.h", "ch_kernels.hip", "ch_plan.h")


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


def measured_traffic():
    """HBM bytes per x-pass launch from the committed counter summary, if it
    was taken on the current kernel sources; otherwise None."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    src = re.search(r"^source-hash:\s*(\w+)", text, re.M)
    val = re.search(r"^traffic-bytes-per-launch:\s*([0-9.eE+]+)", text, re.M)
    if not src or not val or src.group(1) != x_source_hash():
        return None
    return float(val.group(1))


def counter_probe(prec="fp32"):
    """A short run for rocprofv3 counter passes: two steps of the workload
    (FP32 unless `prec` says otherwise), then one device-to-device copy of
    256 MiB (the kernel whose FETCH_SIZE / WRITE_SIZE readings calibrate the
    counters)."""
    import torch
    from paper_2105_01865_amd import ch, inputs
    wl = inputs.make_workload(2)
    stream = torch.cuda.Stream()
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
    advance in one graph launch per step."""
    import numpy as np
    import torch
    from paper_2105_01865_amd import ch, inputs
    E = inputs.ensemble(48)
    pts = sum(w.points for w in E)
    res = {}
    fields = {}
    for prec in ("fp32", "fp64"):
        b = ch.Batch([w.shape for w in E], [w.h for w in E], [w.Cn for w in E],
                     [w.Pe for w in E], stream=stream, precision=prec)
        U, V, W = (b.pack([getattr(w, f) for w in E], f) for f in "uvw")
        b.set_field(b.pack([w.C for w in E], "c"))
        tune = b.autotune(U, V, W, 1e-4, steps=5) if not args.no_autotune else None
        m0 = np.array(b.mass())
        b.step(U, V, W, 1e-4, args.warmup)
        ms = _timed_events(stream, lambda: b.step(U, V, W, 1e-4, args.ensemble_steps))
        m1 = np.array(b.mass())
        fields[prec] = b.get_field().double().cpu().numpy()
        b.profile(True)
        b.step(U, V, W, 1e-4, 5)
        kern = {k: b.profile_read(k) for k in ("x", "y", "z")}
        b.profile(False)
        b.close()
        res[prec] = {"value": round(pts * args.ensemble_steps / (ms * 1e-3) / 1e9, 4),
                     "unit": "Gpts/s", "ms_per_step": round(ms / args.ensemble_steps, 4),
                     "max_box_mass_drift": float(np.max(np.abs(m1 - m0) / np.abs(m0))),
                     "autotune": tune,
                     "kernels_avg_us": {k: round(1e3 * v[0] / max(1, v[1]), 1)
                                        for k, v in kern.items()}}
    d = fields["fp32"] - fields["fp64"]
    return {"workload": "48 periodic boxes, edge ~ U{48,64,96,128,160,192}, h = 1/edge, "
                        "1-20 tanh drops R~U[4,12]h, ABC flow A,B,C~U[0.05,0.2], dt=1e-4",
            "points": pts, "steps": args.ensemble_steps, "fp32": res["fp32"], "fp64": res["fp64"],
            "fp32_over_fp64": round(res["fp32"]["value"] / res["fp64"]["value"], 3),
            "l2_rel_fp32_vs_fp64": float(np.linalg.norm(d) / np.linalg.norm(fields["fp64"]))}


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
            m1 = s.mass()
            if mode == "plain":
                fields[prec] = s.get_field().double().cpu().numpy()
            s.profile(True)
            s.step_multires(ip, UC, VC, WC, wl.dt, 5)
            kern = {k: s.profile_read(k) for k in ("x", "y", "z", "interp")}
            s.profile(False)
            clo = ip.closure()
            s.close()
            ip.close()
            t_us = 1e3 * kern["interp"][0] / max(1, kern["interp"][1])
            r = {"value": round(wl.points * args.multires_steps / (ms * 1e-3) / 1e9, 4),
                 "unit": "Gpts/s", "ms_per_step": round(ms / args.multires_steps, 4),
                 "mass_drift": abs(m1 - m0) / abs(m0), "autotune": tune,
                 "kernels_avg_us": {k: round(1e3 * v[0] / max(1, v[1]), 1)
                                    for k, v in kern.items()}}
            nbytes = transfer_bytes_per_component(uc.shape, wl.shape, es)
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
    d = fields["fp32"] - fields["fp64"]
    return {"workload": "512^3 fine mesh, periodic x,y, no-flux z, 1000 tanh drops R~U[4,12]h; "
                        "velocity on 256x256x192 (tanh-stretched z) transferred every step "
                        "(transfer inside the step time), plain and solenoidal transfer",
            "points": wl.points, "steps": args.multires_steps, "dt": wl.dt,
            "fp32": res["fp32"]["plain"], "fp64": res["fp64"]["plain"],
            "solenoidal": {"fp32": res["fp32"]["solenoidal"], "fp64": res["fp64"]["solenoidal"]},
            "fp32_over_fp64": round(res["fp32"]["plain"]["value"] / res["fp64"]["plain"]["value"], 3),
            "l2_rel_fp32_vs_fp64": float(np.linalg.norm(d) / np.linalg.norm(fields["fp64"]))}


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
    del wl
    torch.cuda.empty_cache()
    pts = 1536 ** 3
    return {"workload": "1536^3 periodic box, FP32 storage, 4000 tanh drops R~U[4,20]h, "
                        "k^-5/3 field 1<=k<=48 rms 1 (inputs generated on the GPU), "
                        "dt from the advective bound",
            "points": pts, "steps": args.large_steps,
            "fp32": {"value": round(pts * args.large_steps / (ms * 1e-3) / 1e9, 4),
                     "unit": "Gpts/s", "ms_per_step": round(ms / args.large_steps, 3),
                     "mass_drift": abs(m1 - m0) / abs(m0),
                     "kernels_avg_us": {k: round(1e3 * v[0] / max(1, v[1]), 1)
                                        for k, v in kern.items()}},
            "plan": cfg, "autotune": tune}


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
                    choices=("fp32", "fp64"),
                    help="two steps and a 256 MiB copy, for rocprofv3 counter runs")
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
                    cells=cells, label_ms=label_ms, tune=tune)

    r32 = timed("fp32")
    progress("256^3 fp32 done")
    r64 = timed("fp64")
    progress("256^3 fp64 done")
    nstep = args.steps
    v32 = pts * nstep / (r32["ms"] * 1e-3) / 1e9
    v64 = pts * nstep / (r64["ms"] * 1e-3) / 1e9

    # accuracy of FP32 against FP64 after warmup + steps
    C32, C64 = r32["C"], r64["C"]
    l2 = float(np.linalg.norm(C32 - C64) / np.linalg.norm(C64))
    drift32 = abs(r32["m1"] - r32["m0"]) / r32["m0"]
    drift64 = abs(r64["m1"] - r64["m0"]) / r64["m0"]
    v32vol = float((C32 >= 0.5).sum()) * h ** 3
    v64vol = float((C64 >= 0.5).sum()) * h ** 3
    vol_err = abs(v32vol - v64vol) / v64vol
    # per-drop volumes (drops matched by their root, the smallest cell index)
    c64 = dict(zip(r64["roots"].tolist(), r64["cells"].tolist()))
    matched = [(c, c64[r]) for r, c in zip(r32["roots"].tolist(), r32["cells"].tolist()) if r in c64]
    dh = np.cbrt(6.0 * r64["cells"] * h ** 3 / np.pi) / (wl.shape[0] * h)
    drops = {"definition": "face-connected cells with C >= 1/2 (periodic), V = h^3 cells, "
                           "(4 pi/3)(D/2)^3 = V, H = box height",
             "count_fp32": int(len(r32["roots"])), "count_fp64": int(len(r64["roots"])),
             "matched_by_root": len(matched),
             "max_rel_volume_err_fp32_vs_fp64": max((abs(a - b) / b for a, b in matched),
                                                    default=None),
             "D_over_H_fp64": {"min": float(dh.min()), "median": float(np.median(dh)),
                               "max": float(dh.max())} if len(dh) else None,
             "label_ms_fp32": round(r32["label_ms"], 2), "label_ms_fp64": round(r64["label_ms"], 2),
             "label_ms_note": "ch_drops wall time: labelling, counting, copy-out and sort",
             "l_loss_fp32": (r32["m1"] - r32["m0"]) / r32["m0"],
             "l_loss_fp64": (r64["m1"] - r64["m0"]) / r64["m0"]}

    def kern(r):
        return {k: dict(avg_us=round(1e3 * r["prof"][k][0] / max(1, r["prof"][k][1]), 2),
                        launches=r["prof"][k][1]) for k in ("x", "y", "z")}

    # roofline of the x pass (FP32 run: the headline precision)
    xms, xn = r32["prof"]["x"]
    x_avg_s = xms / xn * 1e-3
    x_flops = x_pass_flops_per_point() * pts
    achieved = x_flops / x_avg_s / 1e12
    x_bytes = x_pass_bytes_per_point(4) * pts
    x_gbs = x_bytes / x_avg_s / 1e9
    traffic = measured_traffic()

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
        "accuracy_fp32_vs_fp64": {"steps": args.warmup + nstep, "l2_rel": l2,
                                  "mass_drift_fp32": drift32, "mass_drift_fp64": drift64,
                                  "drop_volume_err": vol_err, "drops": drops},
        "hbm_frac_step_model": round(step_bytes_per_point(4) * pts /
                                     (r32["ms"] / nstep * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "alu", "kernel": "k_pass_x (explicit terms + RHS + x solve), fp32",
                     "achieved": round(achieved, 3), "peak": VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 4),
                     "traffic": traffic, "traffic_unit": "HBM bytes per launch (rocprofv3 "
                     "FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "flops_per_point": x_pass_flops_per_point(),
                     "avg_launch_us": round(x_avg_s * 1e6, 2),
                     "hbm_view": {"bytes_per_point": x_pass_bytes_per_point(4),
                                  "achieved_gbs": round(x_gbs, 1),
                                  "frac_of_8000": round(x_gbs / HBM_PEAK_GBS, 4),
                                  # measured bytes (counters) over the same launch time
                                  "measured_gbs": (round(traffic / x_avg_s / 1e9, 1)
                                                   if traffic else None),
                                  "measured_frac_of_8000": (round(traffic / x_avg_s / 1e9
                                                                  / HBM_PEAK_GBS, 4)
                                                            if traffic else None)},
                     "window": f"{args.profile_steps} profiled steps, HIP events per launch"},
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
        line["explicit25"] = bench_explicit25(args, stream, line)
        progress("explicit 25-point done")

    if not args.no_cpu_baseline:
        # the FP64 oracle on the same workload, whole RK3 steps until about
        # 10 s of work (at most 30 s)
        import oracle
        C = wl.C
        steps = 0
        t0 = time.perf_counter()
        while True:
            C = oracle.step(C, wl.u, wl.v, wl.w, h, wl.Cn, wl.Pe, wl.dt, 1)
            steps += 1
            el = time.perf_counter() - t0
            if el >= 10.0 or el / steps * (steps + 1) > 30.0:
                break
        line["cpu_baseline"] = {"value": round(pts * steps / el / 1e9, 6), "unit": "Gpts/s",
                                "cores": oracle.threads(), "kind": "oracle",
                                "sample": f"{steps} RK3 step(s) of the same {wl.shape[2]}^3 "
                                          f"workload in FP64, {el:.1f} s"}
        progress("cpu baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
