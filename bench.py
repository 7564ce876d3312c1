"""Benchmark of the Cahn-Hilliard update on one MI355X.

Workload: the 256^3 periodic box with 64 tanh drops (radii 6-16 h) in a
frozen divergence-free k^-5/3 velocity field (1 <= k <= 16, rms 1),
Cn = h, Pe = 0.9/Cn, dt = 1e-4.  Inputs are seeded and synthetic and are
resident in HBM before the timed region starts.

A step is one full RK3 step (3 substages x {x pass, y solve, z solve}).
`value` is the FP32 throughput in grid-point updates per second (Gpts/s);
the FP64 throughput, the FP32-vs-FP64 error after the timed steps, the
roofline of the dominant kernel (the x pass) and the FP64 CPU oracle's
throughput on a bounded sample are reported on the same JSON line.

    python bench.py [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
METRIC = ("CH grid-point updates/s (Gpts/s) FP32 & batched vs FP64 at stated error; "
          "%HBM peak")


def x_pass_bytes_per_point(s):
    """Algorithmic HBM bytes per grid point of one x-pass launch, averaged over
    the three substages: reads C, u, v, w (+ the old E in substages 2 and 3),
    writes the RHS q (+ the new E in substages 1 and 2): 6s, 7s, 6s."""
    return (6 + 7 + 6) / 3.0 * s


def step_bytes_per_point(s):
    """Algorithmic bytes per point of a whole RK3 step: 34 s (three passes of
    11, 12, 11 element accesses)."""
    return 34.0 * s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=None, help="shrink the box (testing only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library "
              "has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2105_01865_amd import ch, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = inputs.make_workload(2, n=args.n)
    pts = wl.points
    stream = torch.cuda.Stream()
    h = wl.h

    def timed(prec):
        dt_ = torch.float64 if prec == "fp64" else torch.float32
        s = ch.State(wl.shape, h, wl.Cn, wl.Pe, precision=prec, stream=stream)
        C0 = torch.from_numpy(wl.C).to(device="cuda", dtype=dt_)
        U, V, W = (torch.from_numpy(a).to(device="cuda", dtype=dt_) for a in (wl.u, wl.v, wl.w))
        s.set_field(C0)
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
        # the dominant kernel, timed launch by launch with HIP events on the
        # library's stream over a profiled run of the same steps
        s.set_field(C0)
        s.profile(True)
        s.step(U, V, W, wl.dt, args.profile_steps)
        prof = {k: s.profile_read(k) for k in ("x", "y", "z")}
        s.profile(False)
        s.close()
        return dict(ms=ms, wall=wall, m0=m0, m1=m1, C=C, cfg=cfg, prof=prof)

    r32 = timed("fp32")
    r64 = timed("fp64")
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

    # roofline of the x pass (FP32 run: the headline precision)
    xms, xn = r32["prof"]["x"]
    x_avg_s = xms / xn * 1e-3
    x_bytes = x_pass_bytes_per_point(4) * pts
    achieved = x_bytes / x_avg_s / 1e9
    kern = {k: dict(avg_us=1e3 * r32["prof"][k][0] / max(1, r32["prof"][k][1]),
                    launches=r32["prof"][k][1]) for k in ("x", "y", "z")}
    kern64 = {k: dict(avg_us=1e3 * r64["prof"][k][0] / max(1, r64["prof"][k][1]),
                      launches=r64["prof"][k][1]) for k in ("x", "y", "z")}

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
                   "plan": r32["cfg"]},
        "fp64": {"value": round(v64, 4), "unit": "Gpts/s",
                 "ms_per_step": round(r64["ms"] / nstep, 5), "plan": r64["cfg"]},
        "fp32_over_fp64": round(v32 / v64, 3),
        "accuracy_fp32_vs_fp64": {"steps": args.warmup + nstep, "l2_rel": l2,
                                  "mass_drift_fp32": drift32, "mass_drift_fp64": drift64,
                                  "drop_volume_err": vol_err},
        "hbm_frac_step_model": round(step_bytes_per_point(4) * pts /
                                     (r32["ms"] / nstep * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "kernel": "k_pass_x (explicit terms + RHS + x solve)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_point": x_pass_bytes_per_point(4),
                     "avg_launch_us": round(x_avg_s * 1e6, 2),
                     "window": f"{args.profile_steps} profiled steps, HIP events per launch"},
        "kernels_fp32": kern,
        "kernels_fp64": kern64,
    }

    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        oracle.step(wl.C, wl.u, wl.v, wl.w, h, wl.Cn, wl.Pe, wl.dt, 1)
        el = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(pts / el / 1e9, 6), "unit": "Gpts/s",
                                "cores": oracle.threads(), "kind": "oracle",
                                "sample": f"1 RK3 step of the same {wl.shape[2]}^3 workload in "
                                          f"FP64 ({el:.1f} s)"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
