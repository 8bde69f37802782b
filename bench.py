#!/usr/bin/env python3
"""Throughput benchmark of the filtered LB-MHD engine on one MI355X.

Workload (one "step" = one timestep of each run, the whole hot path):
  * LES, 1024 x 1024, filter width Delta = 4 (plain Delta^2/12 closure), FP32;
  * DNS, 4096 x 4096, closure off, FP32;
both the Kelvin-Helmholtz double shear layer U0 = 0.05, delta = L/40,
B0 = 0.01, nu = eta = 2e-4 (MRT ghost rates 1.6), with the FP64 diagnostics (energy, enstrophy,
J_z^2, div B, conservation sums) of both runs every 100 steps inside the
timed region.  Inputs are synthetic (analytic initial state), resident in HBM
before timing starts.

Prints one JSON line: MLUPS (lattice updates of both runs per second), the
HBM roofline of the dominant kernel (the 4096^2 sweep) from HIP events on the
stream the kernels run on, and the FP64 CPU oracle timed on a bounded sample
of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_LUP_FP32 = 38 * 4    # 19 populations read + 19 written per lattice update
KH = dict(U0=0.05, delta_over_L=1.0 / 40.0, B0=0.01, rho0=1.0, pert_amp_over_U0=1e-3, noise_amp=1e-5)
NU = ETA = 2e-4
# MRT ghost rates s5..s8.  At nu = eta = 2e-4 (tau = 0.5006, grid Reynolds number
# U0/nu = 250) the single-relaxation-time collision (ghost rates = s3) grows a
# grid-scale mode and overflows after ~1.5-3.5k steps, on the oracle as on the
# GPU; ghost rates >= 1.4 keep both runs finite for 20000 steps.
GHOST = 1.6
LES_N, LES_DELTA = 1024, 4.0
DNS_N = 4096
KERNEL_SRC = os.path.join(ROOT, "paper_1705_09807_amd", "csrc", "lbmhd_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(kernel: str, lups: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading), or
    None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            m = re.match(r"^\s*([a-z0-9_]+)\s*[:=]\s*(\S+)", line)
            if m:
                vals[m.group(1)] = m.group(2)
    try:
        if vals.get("kernel_source_sha256") != kernel_source_hash():
            return None
        if int(vals["lups_per_launch"]) != lups:
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(les_steps: int, dns_steps: int) -> dict:
    """The FP64 NumPy oracle on a bounded sample of the same workload, one thread."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle.lbmhd_oracle import Oracle

    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        lups = 0
        elapsed = 0.0
        for n, delta, steps in ((LES_N, LES_DELTA, les_steps), (DNS_N, 0.0, dns_steps)):
            if steps <= 0:
                continue
            o = Oracle(n, n, NU, ETA, delta=delta, s5=GHOST, s6=GHOST, s7=GHOST, s8=GHOST)
            o.init_kh_jet(seed=0, **KH)
            t0 = time.perf_counter()
            o.step(steps)
            elapsed += time.perf_counter() - t0
            lups += n * n * steps
            log(f"oracle {n}^2 delta={delta}: {steps} steps in {time.perf_counter() - t0:.2f} s")
            del o
    finally:
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else None
    return {
        "value": lups / elapsed / 1e6,
        "unit": "MLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"FP64 NumPy oracle, 1 thread: {LES_N}^2 LES (Delta={LES_DELTA:g}) x {les_steps} steps "
                  f"+ {DNS_N}^2 DNS x {dns_steps} step(s), {elapsed:.1f} s",
    }


def precision_study(steps: int, dev, stream) -> int:
    """Per-field relative L2 error (rho; m as a vector field; B as a vector
    field) of FP32, FP16 and BF16 storage against an FP64 run of the same
    8192^2 jet, every `steps // 10` steps."""
    import torch

    from paper_1705_09807_amd import Sim

    n, nu, b0 = 8192, 1e-4, 0.01
    kh = dict(KH)
    kh["B0"] = b0
    ghost = dict(s5=GHOST, s6=GHOST, s7=GHOST, s8=GHOST)
    sims = {dt: Sim(nx=n, ny=n, nu=nu, eta=nu, delta=0.0, dtype=dt, b_ref=(b0, 0.0), device=dev, stream=stream,
                    **ghost) for dt in ("fp64", "fp32", "fp16", "bf16")}
    for sim in sims.values():
        sim.init_kh_jet(seed=0, **kh)
    out = {"study": "storage precision vs FP64", "grid": n, "nu": nu, "eta": nu, "B0": b0,
           "mrt_ghost_rates": GHOST, "delta": 0.0, "records": []}
    every = max(1, steps // 10)
    ref = torch.empty((5, n, n), dtype=torch.float64, device=dev)
    cur = torch.empty_like(ref)

    def rel(a, b):
        return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

    done = 0
    while done < steps:
        c = min(every, steps - done)
        for sim in sims.values():
            sim.step(c)
        done += c
        sims["fp64"].moments(ref)
        rec = {"t": done}
        for dt in ("fp32", "fp16", "bf16"):
            sims[dt].moments(cur)
            rec[dt] = {"rho": rel(cur[0], ref[0]), "m": rel(cur[1:3], ref[1:3]), "B": rel(cur[3:5], ref[3:5])}
        d = sims["fp64"].diagnostics()
        rec["fp64_e_kin"], rec["fp64_enstrophy"], rec["fp64_nonfinite"] = d["e_kin"], d["enstrophy"], d["nonfinite"]
        out["records"].append(rec)
        log(json.dumps(rec))
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--les4096-steps", type=int, default=300,
                    help="steps of a supplementary 4096^2 LES timing (0 = skip)")
    ap.add_argument("--lowprec-steps", type=int, default=50,
                    help="steps of the supplementary 8192^2 FP32/FP16/BF16 timings (0 = skip)")
    ap.add_argument("--cpu-les-steps", type=int, default=15)
    ap.add_argument("--cpu-dns-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision-study", type=int, default=0, metavar="STEPS",
                    help="instead of the benchmark: run the 8192^2 jet (nu = eta = 1e-4, B0 = 0.01) "
                         "for STEPS steps in FP64, FP32, FP16 and BF16 storage and print the per-field "
                         "relative L2 errors against the FP64 run as one JSON line")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after timing, run a plain device-to-device copy of this many bytes "
                         "(reference kernel for the HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the sharded design is described in DESIGN.md); use --gpus 1", file=sys.stderr)
        return 2

    import torch

    from paper_1705_09807_amd import Sim

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    log(f"device: {torch.cuda.get_device_name(dev)}")
    if args.precision_study > 0:
        return precision_study(args.precision_study, dev, stream)

    bref = (KH["B0"], 0.0)
    ghost = dict(s5=GHOST, s6=GHOST, s7=GHOST, s8=GHOST)
    les = Sim(nx=LES_N, ny=LES_N, nu=NU, eta=ETA, delta=LES_DELTA, dtype="fp32", schedule="fused",
              b_ref=bref, device=dev, stream=stream, **ghost)
    dns = Sim(nx=DNS_N, ny=DNS_N, nu=NU, eta=ETA, delta=0.0, dtype="fp32", schedule="fused",
              b_ref=bref, device=dev, stream=stream, **ghost)
    les.init_kh_jet(seed=0, **KH)
    dns.init_kh_jet(seed=0, **KH)

    # warmup
    left = args.warmup
    while left > 0:
        c = min(left, args.diag_every)
        dns.step(c)
        les.step(c)
        left -= c
    torch.cuda.synchronize(dev)
    log(f"warmup {args.warmup} steps done")

    K = args.steps
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    chunks = []
    diag_log = []
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    done = 0
    while done < K:
        c = min(args.diag_every, K - done)
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        dns.step(c)
        e1.record(stream)
        les.step(c)
        e2.record(stream)
        chunks.append((c, e0, e1, e2))
        done += c
        if done % args.diag_every == 0:
            diag_log.append((dns.diagnostics(), les.diagnostics()))
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    T = t1 - t0
    dns_ms = sum(e0.elapsed_time(e1) for _, e0, e1, _ in chunks) / K
    les_ms = sum(e1.elapsed_time(e2) for _, _, e1, e2 in chunks) / K
    log(f"timed {K} steps in {T:.3f} s: dns {dns_ms * 1e3:.1f} us/step, les {les_ms * 1e3:.1f} us/step")

    lups_step = LES_N * LES_N + DNS_N * DNS_N
    value = K * lups_step / T / 1e6
    dns_lups = DNS_N * DNS_N
    achieved = BYTES_PER_LUP_FP32 * dns_lups / (dns_ms * 1e-3) / 1e9
    traffic = measured_traffic("fused_dns_fp32", dns_lups)
    roofline = {
        "bound": "hbm",
        "kernel": "k_fused_dns<float> (4096^2 sweep)",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "algorithmic_bytes_per_launch": BYTES_PER_LUP_FP32 * dns_lups,
        "avg_launch_us": round(dns_ms * 1e3, 2),
    }
    les_bw = BYTES_PER_LUP_FP32 * LES_N * LES_N / (les_ms * 1e-3) / 1e9
    extra = {
        "les1024": {"mlups": round(LES_N * LES_N / (les_ms * 1e-3) / 1e6, 1), "avg_launch_us": round(les_ms * 1e3, 2),
                    "algorithmic_GBps": round(les_bw, 1),
                    "note": "state (160 MB) is Infinity-Cache resident: not an HBM figure"},
        "dns4096": {"mlups": round(dns_lups / (dns_ms * 1e-3) / 1e6, 1)},
    }

    if args.les4096_steps > 0:
        del les
        big = Sim(nx=DNS_N, ny=DNS_N, nu=NU, eta=ETA, delta=LES_DELTA, dtype="fp32", schedule="fused",
                  b_ref=bref, device=dev, stream=stream, **ghost)
        big.init_kh_jet(seed=0, **KH)
        big.step(20)
        a, b = ev(), ev()
        a.record(stream)
        big.step(args.les4096_steps)
        b.record(stream)
        torch.cuda.synchronize(dev)
        ms = a.elapsed_time(b) / args.les4096_steps
        bw = BYTES_PER_LUP_FP32 * dns_lups / (ms * 1e-3) / 1e9
        extra["les4096"] = {"mlups": round(dns_lups / (ms * 1e-3) / 1e6, 1), "avg_launch_us": round(ms * 1e3, 2),
                            "achieved_GBps": round(bw, 1), "frac": round(bw / HBM_PEAK_GBS, 4),
                            "kernel": "k_fused_les<float> (plain closure, Delta=4)"}
        log(f"les 4096^2: {ms * 1e3:.1f} us/step, {bw:.0f} GB/s algorithmic")
        del big

    if args.lowprec_steps > 0:
        # 8192^2 jet, nu = eta = 1e-4: storage precision FP32 vs 16-bit deviations
        n8 = 8192
        lups8 = n8 * n8
        kh8 = dict(KH)
        for delta8 in (0.0, LES_DELTA):
            for dt, width in (("fp32", 4), ("fp16", 2), ("bf16", 2)):
                sim8 = Sim(nx=n8, ny=n8, nu=1e-4, eta=1e-4, delta=delta8, dtype=dt, schedule="fused",
                           b_ref=bref, device=dev, stream=stream, **ghost)
                sim8.init_kh_jet(seed=0, **kh8)
                sim8.step(5)
                a, b = ev(), ev()
                a.record(stream)
                sim8.step(args.lowprec_steps)
                b.record(stream)
                torch.cuda.synchronize(dev)
                ms = a.elapsed_time(b) / args.lowprec_steps
                bw = 38 * width * lups8 / (ms * 1e-3) / 1e9
                key = f"{'les' if delta8 else 'dns'}8192_{dt}"
                extra[key] = {"mlups": round(lups8 / (ms * 1e-3) / 1e6, 1), "avg_launch_us": round(ms * 1e3, 2),
                              "bytes_per_lup": 38 * width, "achieved_GBps": round(bw, 1),
                              "frac": round(bw / HBM_PEAK_GBS, 4)}
                log(f"{key}: {ms * 1e3:.1f} us/step, {lups8 / (ms * 1e-3) / 1e6:.0f} MLUPS, {bw:.0f} GB/s")
                del sim8
                torch.cuda.empty_cache()

    last_dns, last_les = diag_log[-1] if diag_log else ({}, {})
    out = {
        "metric": "MLUPS + % HBM roofline",
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(T / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "Kelvin-Helmholtz jet, LES 1024^2 Delta=4 + DNS 4096^2, FP32, "
                        "diagnostics every 100 steps",
            "grids": [LES_N, DNS_N],
            "delta": [LES_DELTA, 0.0],
            "U0": KH["U0"], "delta_over_L": KH["delta_over_L"], "B0": KH["B0"], "nu": NU, "eta": ETA,
            "mrt_ghost_rates": GHOST,
            "diag_every": args.diag_every,
            "schedule": "fused",
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "extra": extra,
        "diagnostics_last": {"dns": {k: last_dns.get(k) for k in ("t", "e_kin", "e_mag", "enstrophy", "j2")},
                             "les": {k: last_les.get(k) for k in ("t", "e_kin", "e_mag", "enstrophy", "j2")}},
        "cpu_baseline": None,
    }
    del dns
    torch.cuda.empty_cache()
    if args.copy_bytes > 0:
        a = torch.empty(args.copy_bytes, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize(dev)
        del a, b
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_les_steps, args.cpu_dns_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
