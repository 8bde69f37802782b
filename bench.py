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
    """SHA-256 (16 hex digits) of the kernel source with comments and blank
    space removed, so an edit of comments alone keeps a counter summary valid
    while any change of code invalidates it."""
    with open(KERNEL_SRC) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    text = re.sub(r"\s+", " ", text).strip()
    return hashlib.sha256(text.encode()).hexdigest()[:16]


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


def host_cpu() -> dict:
    """CPU model (/proc/cpuinfo), os.cpu_count() and the cores this process may
    run on (its affinity mask)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cores": usable}


def _oracle_run(n: int, delta: float, steps: int, seed: int) -> tuple:
    """One single-threaded oracle run of the benchmark jet (worker of the
    all-core leg): lattice updates and seconds."""
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(limits=1)
    except ImportError:  # pragma: no cover
        lim = None
    from oracle.lbmhd_oracle import Oracle

    o = Oracle(n, n, NU, ETA, delta=delta, s5=GHOST, s6=GHOST, s7=GHOST, s8=GHOST)
    o.init_kh_jet(seed=seed, **KH)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    del lim
    return n * n * steps, dt


def cpu_baseline(les_steps: int, dns_steps: int, all_steps: int, max_procs: int = 16) -> dict:
    """The FP64 NumPy oracle on a bounded sample of the same workload: one
    thread (les_steps of the 1024^2 LES + dns_steps of the 4096^2 DNS), and
    all host cores (one single-threaded process per usable core, at most
    max_procs, each running all_steps of the 1024^2 LES on its own seed;
    aggregate = total lattice updates / wall time of the slowest).  Runs
    before the GPU is touched, so the worker processes start from a clean
    parent."""
    import multiprocessing as mp

    host = host_cpu()
    lups = 0
    elapsed = 0.0
    for n, delta, steps in ((LES_N, LES_DELTA, les_steps), (DNS_N, 0.0, dns_steps)):
        if steps <= 0:
            continue
        l, dt = _oracle_run(n, delta, steps, 0)
        lups += l
        elapsed += dt
        log(f"oracle {n}^2 delta={delta}: {steps} steps in {dt:.2f} s")
    out = {
        "value": lups / elapsed / 1e6,
        "unit": "MLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"FP64 NumPy oracle, 1 thread: {LES_N}^2 LES (Delta={LES_DELTA:g}) x {les_steps} steps "
                  f"+ {DNS_N}^2 DNS x {dns_steps} step(s), {elapsed:.1f} s",
        **host,
    }
    procs = max(1, min(max_procs, host["affinity_cores"]))
    if all_steps > 0 and procs > 1:
        ctx = mp.get_context("spawn")
        t0 = time.perf_counter()
        with ctx.Pool(procs) as pool:
            res = pool.starmap(_oracle_run, [(LES_N, LES_DELTA, all_steps, k) for k in range(procs)])
        wall = time.perf_counter() - t0
        tot = sum(r[0] for r in res)
        slowest = max(r[1] for r in res)
        out.update({
            "cores_all": procs,
            "mlups_all": tot / slowest / 1e6,
            "sample_all": f"{procs} single-threaded FP64 oracle processes, each {LES_N}^2 LES "
                          f"(Delta={LES_DELTA:g}) x {all_steps} steps on its own seed; slowest {slowest:.1f} s "
                          f"({wall:.1f} s with process start)",
        })
        log(f"oracle on {procs} cores: {out['mlups_all']:.1f} MLUPS aggregate")
    return out


def variant_oracle_rates(n: int = 512, steps: int = 2) -> dict:
    """The FP64 oracle, one thread, on an n^2 sample (`steps` steps of the
    same jet) in the mode that matches each closure / lattice variant the
    benchmark times on the GPU, in MLUPS.  The in-place synchronous schedule
    computes the same step as the fused one and the storage types are not
    emulated, so those legs share the plain oracle's rate."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import numpy as np
    from oracle.lbmhd_oracle import Oracle
    from oracle import learned as OL

    def learned_hook():
        # a seeded random network (the oracle's cost per cell does not depend
        # on the weights); the pad row of w1 is zero
        rng = np.random.default_rng(0)
        nm = {"w1": rng.normal(0.0, 0.125, (64, 64)), "b1": rng.normal(0.0, 0.01, 64),
              "w2": rng.normal(0.0, 0.125, (64, 64)), "b2": rng.normal(0.0, 0.01, 64),
              "w3": rng.normal(0.0, 0.125, (64, 4)), "b3": rng.normal(0.0, 0.01, 4)}
        nm["w1"][63] = 0.0
        # per-feature normalisation: each field's value on its nine patch columns, pad 0 / 1
        shift = np.append(np.repeat([1.0, 0.0, 0.0, KH["B0"], 0.0, 0.0, 0.0], 9), 0.0)
        scale = np.append(np.repeat([1e3, 20.0, 20.0, 100.0, 100.0, 1e3, 1e3], 9), 1.0)
        return OL.learned_correction(nm, shift, scale, np.full(4, 1e-6))

    modes = {
        "les4096": dict(delta=LES_DELTA),
        "les4096_full": dict(delta=LES_DELTA, density_gradients=True),
        "les4096_local_iso9": dict(delta=LES_DELTA, grad_stencil="local_iso9"),
        "les4096_aa_lagged": dict(delta=LES_DELTA, closure_time="lagged"),
        "les4096_d2q9": dict(delta=LES_DELTA, mag_lattice="d2q9"),
        "dns4096_d2q9": dict(delta=0.0, mag_lattice="d2q9"),
        "les1024_learned": dict(delta=LES_DELTA, closure_correction="learned"),
    }
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    out = {}
    try:
        for key, kw in modes.items():
            kw = dict(kw)
            if kw.get("closure_correction") == "learned":
                kw["closure_correction"] = learned_hook()
            o = Oracle(n, n, NU, ETA, s5=GHOST, s6=GHOST, s7=GHOST, s8=GHOST, **kw)
            o.init_kh_jet(seed=0, **KH)
            t0 = time.perf_counter()
            o.step(steps)
            dt = time.perf_counter() - t0
            out[key] = {"oracle_mlups": round(n * n * steps / dt / 1e6, 3),
                        "oracle_sample": f"FP64 NumPy oracle, 1 thread, {n}^2 x {steps} steps, {dt:.2f} s"
                                         + ("; network evaluated every step" if "closure_correction" in kw else "")}
            log(f"oracle {key}: {dt:.2f} s")
    finally:
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else None
    return out


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


JET_RUNS = {
    # label: (grid, Delta, nu = eta, length in units of the LES run's steps)
    "dns1024": (1024, 0.0, 1e-3, 1),
    "les1024_d1": (1024, 1.0, 1e-3, 1),
    "les1024_d2": (1024, 2.0, 1e-3, 1),
    "dns2048": (2048, 0.0, 2e-3, 2),
}


def _slope(ek, lo, hi):
    """Least-squares exponent a of E(k) ~ k^a over the integer bins lo..hi."""
    import numpy as np
    k = np.arange(lo, hi + 1, dtype=np.float64)
    e = np.asarray(ek[lo:hi + 1], dtype=np.float64)
    ok = e > 0
    return float(np.polyfit(np.log(k[ok]), np.log(e[ok]), 1)[0])


def jet_compare(spectra: dict, a: str, b: str, kmax: int = 128) -> dict:
    """Relative L2 distance of the total-energy spectra E_K + E_M of run a at
    LES time t and run b at its matching time (2t for DNS 2048^2 against a
    1024^2 run), over the bins 1..kmax, for every common snapshot."""
    import numpy as np
    ma, mb = JET_RUNS[a][3], JET_RUNS[b][3]
    out = {}
    for ta, sa in spectra.get(a, {}).items():
        tb = str(int(ta) * mb // ma)
        sb = spectra.get(b, {}).get(tb)
        if sb is None:
            continue
        ea = np.asarray(sa["E_K"][1:kmax + 1]) + np.asarray(sa["E_M"][1:kmax + 1])
        eb = np.asarray(sb["E_K"][1:kmax + 1]) + np.asarray(sb["E_M"][1:kmax + 1])
        out[f"{ta}/{tb}"] = round(float(np.linalg.norm(ea - eb) / np.linalg.norm(eb)), 4)
    return out


def jet_study(args, dev, stream) -> int:
    """The magnetized Kelvin-Helmholtz jet of Sec. 4 on the paper's grids.

    sech^2 jet U0 = 4.88e-2, B_y = B0 = 0.005 U0 along the jet, the four 1 %
    perturbations (lbm_init_sech2_jet); Re = U0 L / nu = 50k at every grid:
    nu = eta = 1e-3 at 1024^2, 2e-3 at 2048^2.  Runs: DNS 1024^2, LES 1024^2
    with Delta = 1 and Delta = 2 (simplified closure of Sec. 3, 3x3 isotropic
    gradients) for T steps, DNS 2048^2 for 2T (t_DNS = 2 t_LES); the paper's
    T is 780k.  Single-relaxation-time collisions (ghost rates = s3), FP64 by
    default: the initial state is periodic in y with period L/4, and FP32
    storage rounds the sub-ulp differences between the four periods away,
    so the vortex-pairing modes are never seeded and the L/4 street never
    merges; in FP64 they grow from round-off.  Reported per run at T/4, T/2 and T (DNS 2048^2: twice those
    steps), and every --jet-every steps when given: kinetic and magnetic energy, enstrophy, max |div B|, and the
    exponent of a power-law fit of the total-energy spectrum E_K + E_M over
    two wavenumber ranges; the paper quotes -1.66 for the 1024^2 runs and
    -1.71 for DNS 2048^2 at the final time (its fit range is not stated).
    One JSON line on stdout; with --out-dir the spectra of every snapshot go
    to <out-dir>/jet_spectra_<variant>_<runs>.json.
    """
    import numpy as np
    import torch

    from paper_1705_09807_amd import Sim
    from paper_1705_09807_amd import learned as G

    T = int(args.jet_study)
    labels = [r for r in args.jet_runs.split(",") if r]
    for r in labels:
        if r not in JET_RUNS:
            log(f"unknown run {r}; choose from {sorted(JET_RUNS)}")
            return 2
    U0 = 4.88e-2
    B0 = 0.005 * U0
    dtype = args.jet_dtype
    # "paper" variant: g on D2Q9 and the closure with the filtered-density
    # terms (Sec. 2's lattice and Sec. 2.1's closure before Sec. 3's
    # simplification); "default": D2Q5 g, simplified closure
    variant = dict(mag_lattice="d2q9", closure="full") if args.jet_variant == "paper" else {}
    out = {"study": "sech2 jet (Sec. 4)", "variant": args.jet_variant, "T_les": T, "U0": U0, "B0": B0, "Re": 5e4,
           "dtype": dtype,
           "collision": "SRT", "runs": {}}
    spectra = {}
    for label in labels:
        n, delta, nu, mult = JET_RUNS[label]
        steps = T * mult
        sim = Sim(nx=n, ny=n, nu=nu, eta=nu, delta=delta, dtype=dtype, b_ref=(0.0, B0), device=dev, stream=stream,
                  **variant)
        sim.init_sech2_jet(U0=U0, B0=B0, pert=0.01, k=4)
        marks = {steps // 4, steps // 2, steps}
        if args.jet_every > 0:  # and every jet_every LES steps (scaled like the run's time)
            marks |= set(range(args.jet_every * mult, steps + 1, args.jet_every * mult))
        marks = sorted(marks)
        rec = {"grid": n, "delta": delta, "nu": nu, "eta": nu, "steps": steps, "snapshots": {}}
        chunk = max(1, min(20000 * mult, steps // 8))
        t0 = time.perf_counter()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        gpu_ms = 0.0
        while sim.t < steps:
            nxt = min(steps, sim.t + chunk, min(m for m in marks if m > sim.t))
            ev0.record(stream)
            sim.step(nxt - sim.t)
            ev1.record(stream)
            torch.cuda.synchronize(dev)
            gpu_ms += ev0.elapsed_time(ev1)
            d = sim.diagnostics()
            log(f"{label}: t = {sim.t} e_kin {d['e_kin']:.6e} e_mag {d['e_mag']:.6e} "
                f"nonfinite {d['nonfinite']} ({time.perf_counter() - t0:.0f} s)")
            if d["nonfinite"] or not np.isfinite(d["e_kin"]):
                rec["overflow_at"] = sim.t
                break
            if sim.t in marks:
                ek, em, _ = G.spectra(sim.moments())
                tot = (ek + em).cpu().numpy()
                snap = {k: d[k] for k in ("e_kin", "e_mag", "enstrophy", "j2", "divb_max", "divb_rms")}
                snap["slope_k8_64"] = round(_slope(tot, 8, 64), 3)
                snap["slope_k16_128"] = round(_slope(tot, 16, 128), 3)
                snap["slope_k8_64_kinetic"] = round(_slope(ek.cpu().numpy(), 8, 64), 3)
                rec["snapshots"][str(sim.t)] = snap
                spectra.setdefault(label, {})[str(sim.t)] = {"E_K": ek.cpu().tolist(), "E_M": em.cpu().tolist()}
        rec["gpu_seconds"] = round(gpu_ms / 1e3, 2)
        rec["mlups"] = round(n * n * sim.t / max(gpu_ms, 1e-9) / 1e3, 1)
        out["runs"][label] = rec
        sim.close()
        del sim
        torch.cuda.empty_cache()
    for a in ("les1024_d2", "les1024_d1", "dns1024"):
        if a in spectra and "dns2048" in spectra:
            out[f"spectrum_rel_l2_{a}_vs_dns2048"] = jet_compare(spectra, a, "dns2048")
    if args.out_dir:
        os.makedirs(args.out_dir, exist_ok=True)
        with open(os.path.join(args.out_dir, f"jet_spectra_{args.jet_variant}_{'_'.join(labels)}.json"), "w") as fh:
            json.dump(spectra, fh)
    print(json.dumps(out), flush=True)
    return 0


def _study_setup(args):
    """The learned-closure study's jet and grids (training.JetSetup)."""
    from paper_1705_09807_amd import training as TR

    # nu = 1e-4, eta = 1e-2 on the LES grid (x4 for the DNS), shear layers
    # of thickness L/100 with modes at 2 % of U0: a jet whose small scales
    # the LES without closure gets wrong by ~20 % in the band N/16 < k <= N/4
    # while the analytic closure stays near 1 %.  With the single-relaxation-
    # time magnetic distribution, runs at eta <= 3e-3 (s_m >= 1.96) overflow
    # at roll-up on both grids (div B grows first); eta = 1e-2 keeps them
    # finite.
    return TR.JetSetup(n_fine=4096, factor=args.study_factor, delta_fine=4.0 * args.study_factor,
                       nu_les=args.study_nu, eta_les=args.study_eta,
                       ghost=GHOST,
                       U0=KH["U0"],
                       delta_over_L=args.study_delta_over_l, B0=KH["B0"], noise_amp=1e-4,
                       modes=(2, 3, 4, 5, 6), mode_amp=args.study_mode_amp)


def _train_study_network(args, setup, t_end: int, dev, stream):
    """Train the network on filtered DNS of seeds 1 and 2 at six LES times up
    to t_end, with the library's kernels.  Returns (mlp, times, losses), or
    (None, ...) when the DNS overflowed."""
    import torch

    from paper_1705_09807_amd import learned as G
    from paper_1705_09807_amd import training as TR

    train_times = [t_end * k // 6 for k in range(1, 7)]
    t0 = time.perf_counter()
    X, T = TR.samples(setup, seeds=[1, 2], les_times=train_times,
                      progress=lambda sd, tt: log(f"samples: seed {sd} LES time {tt} ({time.perf_counter() - t0:.0f} s)"))
    log(f"samples {tuple(X.shape)} in {time.perf_counter() - t0:.1f} s")
    if not (bool(torch.isfinite(X).all()) and bool(torch.isfinite(T).all())):
        log("training samples are not finite: the DNS overflowed")
        return None, train_times, None
    mlp = G.Mlp(G.glorot_params(0), device=dev, stream=stream)
    mlp.fit_norm(X, T)
    t1 = time.perf_counter()
    losses = TR.train(mlp, X, T, steps=args.train_steps, batch=8192, lr=2e-3)
    torch.cuda.synchronize(dev)
    log(f"trained {args.train_steps} steps in {time.perf_counter() - t1:.1f} s: loss {losses[0].item():.3e} -> "
        f"{losses[-200:].mean().item():.3e}")
    del X, T
    torch.cuda.empty_cache()
    return mlp, train_times, losses


def learned_study(args, dev, stream) -> int:
    """A-posteriori test of the learned closure (filtered DNS -> F x coarser
    LES, F = --study-factor, 4 by default).

    DNS 4096^2 (FP32) of the jet at nu_DNS = F nu_LES (constant Reynolds
    number), Gaussian filter of width 4 F fine cells, subsampled every F-th
    cell to (4096 / F)^2 (Delta = 4 LES cells).  The network is trained on two seeds with the
    library's kernels; on a held-out seed the LES (no closure, analytic
    closure and analytic plus learned correction, each with FP32 and FP16
    storage; learned with BF16 storage; learned with the network every
    --corr-every steps) starts from the filtered DNS initial state and runs
    alongside the DNS.  Reported: the relative L2 error of the total-energy
    spectrum E_K + E_M against the filtered DNS over the bins 1 .. N_LES/4 and
    over the small-scale band N_LES/16 < k <= N_LES/4, at several times, the
    growth rate of the streamwise k_x = 3 mode, a-priori subgrid errors, and
    wall-clock throughput of each run.  One JSON line on stdout.
    """
    import math

    import numpy as np
    import torch

    from paper_1705_09807_amd import Sim
    from paper_1705_09807_amd import learned as G
    from paper_1705_09807_amd import training as TR

    setup = _study_setup(args)
    T_END = args.learned_study
    mlp, train_times, losses = _train_study_network(args, setup, T_END, dev, stream)
    if mlp is None:
        return 1

    seed = 3
    dns = TR.dns(setup, seed)
    c0 = TR.filtered(setup, dns)
    K = args.corr_every
    # no closure (Delta = 0: the filtered initial state run as a DNS of the
    # coarse grid), the analytic closure and the analytic plus learned closure
    runs = {"noclosure_fp32": ("none", "fp32", 1), "analytic_fp32": ("analytic", "fp32", 1),
            "learned_fp32": ("learned", "fp32", 1), "noclosure_fp16": ("none", "fp16", 1),
            "analytic_fp16": ("analytic", "fp16", 1), "learned_fp16": ("learned", "fp16", 1),
            "learned_bf16": ("learned", "bf16", 1)}
    if K > 1:
        runs[f"learned_fp32_every{K}"] = ("learned", "fp32", K)
        runs[f"learned_fp16_every{K}"] = ("learned", "fp16", K)
    les = {}
    for name, (closure, dt, every_k) in runs.items():
        g = setup.ghost
        s = Sim(nx=setup.n_les, ny=setup.n_les, nu=setup.nu_les, eta=setup.eta,
                delta=0.0 if closure == "none" else setup.delta_les, s5=g, s6=g, s7=g, s8=g, dtype=dt,
                b_ref=(setup.B0, 0.0), closure="analytic" if closure == "none" else closure, device=dev,
                stream=stream)
        s.init_from_moments(c0[:5].contiguous())
        if closure == "learned":
            s.set_closure_mlp(mlp.pack())
            s.set_correction_interval(every_k)
        les[name] = s
    every = max(T_END // 40, 1)
    n_cmp = setup.n_les // 4
    series = {"t": [], "fdns": []}      # streamwise energy E_x(m), m = 0 .. 8
    for name in runs:
        series[name] = []
    spec_err = {name: [] for name in runs}
    spec_bin = {name: [] for name in runs}      # mean per-bin |E_les / E_fdns - 1| over bins above 1e-10 of the total
    spec_band = {name: [] for name in runs}     # relative L2 over the small-scale band N/16 < k <= N/4
    k_band = setup.n_les // 16
    spectra_at = {"fdns": {}}
    for name in runs:
        spectra_at[name] = {}
    apriori = []
    wall = {name: 0.0 for name in runs}
    wall["dns"] = 0.0
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    t = 0
    while True:
        c = TR.filtered(setup, dns)
        ek, em, ekx = G.spectra(c[:5].contiguous())
        e_f = (ek + em)[1:n_cmp + 1]
        series["t"].append(t)
        series["fdns"].append(ekx[:9].tolist())
        for name, s in les.items():
            mk, mm, mx_ = G.spectra(s.moments())
            series[name].append(mx_[:9].tolist())
            if t > 0 and t % (T_END // 8) == 0:
                e_l = (mk + mm)[1:n_cmp + 1]
                spec_err[name].append((t, (torch.linalg.norm(e_l - e_f) / torch.linalg.norm(e_f)).item()))
                keep = e_f > 1e-10 * e_f.sum()
                spec_bin[name].append((t, (e_l[keep] / e_f[keep] - 1.0).abs().mean().item()))
                spec_band[name].append((t, (torch.linalg.norm(e_l[k_band:] - e_f[k_band:])
                                            / torch.linalg.norm(e_f[k_band:])).item()))
                spectra_at[name][t] = e_l.tolist()
                spectra_at["fdns"][t] = e_f.tolist()
        if t > 0 and t % (T_END // 8) == 0:
            Xs, Ts = G.closure_samples(c, setup.delta_les)
            ana, lea, ood = TR.closure_errors(mlp, Xs, Ts)
            apriori.append((t, (lea.sum() / ana.sum()).item(), ood.item()))
        if t >= T_END:
            break
        if (t // every) % 10 == 0:
            log(f"study t={t}: E_x(3) fdns {series['fdns'][-1][3]:.3e}, "
                + ", ".join(f"{k} {series[k][-1][3]:.3e}" for k in runs))
        a, b = ev(), ev()
        a.record(stream)
        dns.step(every * setup.factor)
        b.record(stream)
        for name, s in les.items():
            x0, x1 = ev(), ev()
            x0.record(stream)
            s.step(every)
            x1.record(stream)
            torch.cuda.synchronize(dev)
            wall[name] += x0.elapsed_time(x1)
        torch.cuda.synchronize(dev)
        wall["dns"] += a.elapsed_time(b)
        t += every
    finite = {name: s.diagnostics()["nonfinite"] == 0 for name, s in les.items()}

    def growth(vals, m=3):
        """Growth rate of the k_x = m amplitude, sqrt(E_x(m)), fitted over the
        snapshots whose energy lies between 1e-3 and 1e-1 of the series peak."""
        v = np.asarray([e[m] for e in vals])
        tt = np.asarray(series["t"], dtype=np.float64)
        peak = v.max()
        m = (v > 1e-3 * peak) & (v < 1e-1 * peak) & (tt > 0)
        if m.sum() < 3:
            m = (tt > 0) & (v < 0.3 * peak)
        if m.sum() < 2:
            return None
        return float(0.5 * np.polyfit(tt[m], np.log(v[m]), 1)[0])

    g_f = growth(series["fdns"])
    res = {}
    for name in runs:
        g_l = growth(series[name])
        res[name] = {
            "spectrum_rel_l2": [(tt, round(e, 6)) for tt, e in spec_err[name]],
            "spectrum_mean_bin_rel_err": [(tt, round(e, 6)) for tt, e in spec_bin[name]],
            "spectrum_band_rel_l2": [(tt, round(e, 6)) for tt, e in spec_band[name]],
            "growth_rate": g_l,
            "growth_rate_rel_err": (None if g_l is None or not g_f else round(g_l / g_f - 1.0, 5)),
            "finite": finite[name],
            "les_ms_per_les_step": round(wall[name] / T_END, 4),
            "fine_equivalent_mlups": round(setup.n_fine ** 2 * setup.factor * T_END / (wall[name] * 1e-3) / 1e6, 1),
        }
    out = {
        "study": "learned closure vs analytic closure against filtered DNS (a posteriori)",
        "dns": f"{setup.n_fine}^2 FP32, nu={setup.nu_dns:g}, eta={setup.eta_dns:g}, {T_END * setup.factor} steps",
        "les": f"{setup.n_les}^2, Delta={setup.delta_les:g}, nu={setup.nu_les:g}, eta={setup.eta:g}, {T_END} steps",
        "filter": f"Gaussian width {setup.delta_fine:g} fine cells, every {setup.factor}th cell",
        "jet": setup.kh(seed),
        "train": {"seeds": [1, 2], "les_times": train_times, "steps": args.train_steps, "batch": 8192,
                  "loss_first": losses[0].item(), "loss_last200": losses[-200:].mean().item()},
        "held_out_seed": seed,
        "spectrum_bins": [1, n_cmp],
        "spectrum_band_bins": [k_band + 1, n_cmp],
        "growth_rate_fdns": g_f,
        "dns_fine_mlups": round(setup.n_fine ** 2 * setup.factor * T_END / (wall["dns"] * 1e-3) / 1e6, 1),
        "apriori_mse_ratio_learned_over_analytic": [(tt, round(r, 4), round(o, 5)) for tt, r, o in apriori],
        "runs": res,
        "series_ex": {k: vals for k, vals in series.items()},
        "spectra_total_bins_1_to_ncmp": spectra_at,
    }
    print(json.dumps(out), flush=True)
    return 0


def production_run(args, dev, stream) -> int:
    """The production configuration run: a 16384^2 jet (268 M cells), nu =
    5e-5, Delta = 4, B = (B0, 0) with B0 = --production-b0, for
    --production-run steps; by default the learned closure, FP16 population
    storage and eta = 5e-5 (--production-closure, --production-dtype,
    --production-eta).  Diagnostics (energies, enstrophy, integral J_z^2,
    div B) and the radially binned kinetic and magnetic spectra with the
    streamwise spectrum E_x(m) every --production-every steps; the run stops
    at the first snapshot with a non-finite value.

    The jet is the learned-closure study's (shear layers U0 = 0.05 of
    thickness L/100, modes 2-6 at 2 % of U0 with seeded phases, noise 1e-4),
    and so is the network: trained first, with the library's kernels, on
    filtered DNS of that jet at the same B0 (4096^2 -> 1024^2; no filtered
    DNS of the 16384^2 jet fits one GPU).  Each snapshot of a learned run
    also records the share of cells whose inputs lie outside the training
    range (the analytic closure alone there) and the RMS of the four
    correction planes.  FP16 is the 16-bit storage that keeps the growth rate
    within 2 % of the filtered DNS in that study; BF16 misses it by 20-33 %.
    Reported: the series, fitted growth rates of E_x(m), m = 1..8, over the
    finite snapshots (where E_x(m) lies between 1e-3 and 1e-1 of its largest
    value, else all snapshots up to that value), and the step time; with
    --out-dir the spectra go to <out-dir>/production_spectra_B0_<B0>_eta_
    <eta>_<closure>_<dtype>.npz.  One JSON line on stdout.
    """
    import numpy as np
    import torch

    from paper_1705_09807_amd import Sim
    from paper_1705_09807_amd import learned as G
    from paper_1705_09807_amd import training as TR

    n, b0, T, every = 16384, args.production_b0, args.production_run, args.production_every
    # the study's jet with this run's field: the network is trained at the
    # same B0 (its normalised inputs would otherwise all lie outside the
    # training range)
    prod = TR.JetSetup(**{**_study_setup(args).__dict__, "B0": b0})
    mlp, losses, packed = None, None, None
    if args.production_closure == "learned":
        mlp, _, losses = _train_study_network(args, prod, 8000, dev, stream)
        if mlp is None:
            return 1
        packed = mlp.pack()
    t0 = time.perf_counter()
    mom0 = TR.jet_fields(prod, n, seed=3, device=dev)
    log(f"initial fields in {time.perf_counter() - t0:.1f} s")
    eta, closure, dtype = args.production_eta, args.production_closure, args.production_dtype
    sim = Sim(nx=n, ny=n, nu=5e-5, eta=eta, delta=LES_DELTA, dtype=dtype, schedule="fused",
              b_ref=(b0, 0.0), closure=closure, device=dev, stream=stream,
              s5=GHOST, s6=GHOST, s7=GHOST, s8=GHOST)
    sim.init_from_moments(mom0)
    del mom0
    torch.cuda.empty_cache()
    learned = closure == "learned"
    if learned:
        sim.set_closure_mlp(packed)
    mom = torch.empty((5, n, n), dtype=torch.float64, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    corr = torch.empty((4, n, n), dtype=torch.float32, device=dev)
    series = {"t": [], "e_kin": [], "e_mag": [], "enstrophy": [], "j2": [], "divb_max": [], "nonfinite": [],
              "ex_m0_to_8": [], "out_of_range_share": [], "correction_rms": []}
    spectra_k, spectra_m, step_ms, spec_ms = [], [], 0.0, 0.0
    t_wall = time.perf_counter()
    while True:
        ev0.record(stream)
        sim.moments(mom)
        ek, em, ekx = G.spectra(mom, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize(dev)
        spec_ms += ev0.elapsed_time(ev1)
        d = sim.diagnostics()
        series["t"].append(sim.t)
        for k in ("e_kin", "e_mag", "enstrophy", "j2", "divb_max", "nonfinite"):
            series[k].append(d[k])
        series["ex_m0_to_8"].append(ekx[:9].tolist())
        # share of cells left to the analytic closure, and the correction's size
        if learned:
            sim.closure_correction(corr)
            torch.cuda.synchronize(dev)
            series["out_of_range_share"].append((corr == 0).all(dim=0).float().mean().item())
            series["correction_rms"].append([torch.linalg.vector_norm(corr[i], dtype=torch.float64).item() / n
                                             for i in range(4)])
        spectra_k.append(ek.float().cpu().numpy())
        spectra_m.append(em.float().cpu().numpy())
        log(f"production B0={b0}: t = {sim.t} e_kin {d['e_kin']:.6e} e_mag {d['e_mag']:.6e} "
            f"E_x(3) {ekx[3].item():.3e} divB_max {d['divb_max']:.2e} nonfinite {d['nonfinite']} "
            + (f"out of range {series['out_of_range_share'][-1]:.3%} " if learned else "")
            + f"({time.perf_counter() - t_wall:.0f} s)")
        if d["nonfinite"] or sim.t >= T:
            break
        ev0.record(stream)
        sim.step(min(every, T - sim.t))
        ev1.record(stream)
        torch.cuda.synchronize(dev)
        step_ms += ev0.elapsed_time(ev1)
    fin = np.asarray(series["nonfinite"]) == 0
    tt = np.asarray(series["t"], dtype=np.float64)[fin]
    ex = np.asarray(series["ex_m0_to_8"])[fin]
    rates = {}
    for m in range(1, 9):
        v = ex[:, m]
        peak = int(np.argmax(v))
        sel = (v > 1e-3 * v[peak]) & (v < 1e-1 * v[peak]) & (np.arange(len(v)) <= peak)
        if sel.sum() < 3:
            sel = np.arange(len(v)) <= peak
        rates[m] = (float(0.5 * np.polyfit(tt[sel], np.log(v[sel]), 1)[0]) if sel.sum() >= 2 and (v[sel] > 0).all()
                    else None)
    steps_done = int(series["t"][-1])
    out = {
        "study": f"production configuration: 16384^2 jet, {closure} closure, {dtype} storage",
        "grid": n, "nu": 5e-5, "eta": eta, "Delta": LES_DELTA, "B0": b0, "steps": steps_done,
        "jet": prod.kh(3) | {"modes": list(prod.modes), "mode_amp_over_U0": prod.mode_amp},
        "network": ({"trained_on": "filtered DNS 4096^2 -> 1024^2 of the same jet (same B0), seeds 1 and 2",
                     "loss_first": losses[0].item(), "loss_last200": losses[-200:].mean().item()}
                    if learned else None),
        "finite": series["nonfinite"][-1] == 0,
        "step_ms": round(step_ms / max(steps_done, 1), 4),
        "mlups": round(n * n * steps_done / max(step_ms, 1e-9) / 1e3, 1),
        "spectra_ms_each": round(spec_ms / len(series["t"]), 2),
        "growth_rate_ex_m": rates,
        "series": series,
    }
    if args.out_dir:
        os.makedirs(args.out_dir, exist_ok=True)
        np.savez_compressed(os.path.join(args.out_dir, f"production_spectra_B0_{b0:g}_eta_{eta:g}_{closure}_{dtype}.npz"),
                            t=np.asarray(series["t"], dtype=np.float64),
                            e_kin=np.stack(spectra_k), e_mag=np.stack(spectra_m))
    sim.close()
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
    ap.add_argument("--learned-steps", type=int, default=300,
                    help="steps of the supplementary 1024^2 learned-closure LES timing (0 = skip)")
    ap.add_argument("--corr-every", type=int, default=16,
                    help="learned-closure legs and study: also time/run with the network evaluated every "
                         "this many steps and its correction held in between (1 = only every step)")
    ap.add_argument("--production-steps", type=int, default=5,
                    help="steps of the supplementary 16384^2 learned-closure timings, BF16 and FP16; with "
                         "the network every --corr-every steps rounded up to whole intervals (0 = skip)")
    ap.add_argument("--cpu-les-steps", type=int, default=15)
    ap.add_argument("--cpu-dns-steps", type=int, default=3)
    ap.add_argument("--cpu-all-steps", type=int, default=20,
                    help="steps of the 1024^2 LES per process in the all-core oracle leg (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision-study", type=int, default=0, metavar="STEPS",
                    help="instead of the benchmark: run the 8192^2 jet (nu = eta = 1e-4, B0 = 0.01) "
                         "for STEPS steps in FP64, FP32, FP16 and BF16 storage and print the per-field "
                         "relative L2 errors against the FP64 run as one JSON line")
    ap.add_argument("--learned-study", type=int, default=0, metavar="LES_STEPS",
                    help="instead of the benchmark: train the learned closure on filtered 4096^2 DNS and "
                         "compare learned and analytic LES (1024^2, or 4096/--study-factor) with the filtered "
                         "DNS of a held-out seed "
                         "over LES_STEPS steps (one JSON line)")
    ap.add_argument("--jet-study", type=int, default=0, metavar="T",
                    help="instead of the benchmark: the magnetized sech^2 jet of the paper, LES runs of T "
                         "steps (the paper's T is 780000) and DNS 2048^2 of 2T (one JSON line)")
    ap.add_argument("--jet-runs", default="dns1024,les1024_d1,les1024_d2,dns2048",
                    help="comma-separated subset of the jet study's runs")
    ap.add_argument("--jet-every", type=int, default=0, metavar="STEPS",
                    help="jet study: also take spectra every STEPS LES steps (twice that for DNS 2048^2)")
    ap.add_argument("--jet-dtype", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--jet-variant", default="default", choices=["default", "paper"],
                    help="paper: D2Q9 magnetic distribution and the density-gradient closure")
    ap.add_argument("--production-run", type=int, default=0, metavar="STEPS",
                    help="run the production configuration (16384^2, learned closure, FP16 storage) for STEPS "
                         "steps at B0 = --production-b0 and report its series; nothing else is run")
    ap.add_argument("--production-b0", type=float, default=0.02)
    ap.add_argument("--production-eta", type=float, default=5e-5,
                    help="production run: resistivity (5e-5 as configured; the single-relaxation-time magnetic "
                         "collision is then at s_m = 1.9994)")
    ap.add_argument("--production-closure", default="learned", choices=["learned", "analytic"])
    ap.add_argument("--production-dtype", default="fp16", choices=["fp16", "bf16", "fp32"])
    ap.add_argument("--production-every", type=int, default=1000,
                    help="production run: spectra and diagnostics every this many steps")
    ap.add_argument("--train-steps", type=int, default=4000)
    ap.add_argument("--study-nu", type=float, default=1e-4, help="LES-grid viscosity of the study")
    ap.add_argument("--study-eta", type=float, default=1e-2, help="LES-grid resistivity of the study")
    ap.add_argument("--study-delta-over-l", type=float, default=1.0 / 100.0,
                    help="shear-layer thickness of the learned-closure study's jet, in units of L")
    ap.add_argument("--study-mode-amp", type=float, default=0.02,
                    help="amplitude of each streamwise mode of the study's jet, in units of U0")
    ap.add_argument("--study-factor", type=int, default=4, choices=[2, 4, 8],
                    help="coarsening of the learned-closure study (LES grid 4096 / factor)")
    ap.add_argument("--out-dir", default="", help="folder for the jet study's per-snapshot spectra")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after timing, run a plain device-to-device copy of this many bytes "
                         "(reference kernel for the HBM byte counters)")
    args = ap.parse_args()
    if args.corr_every < 1:
        ap.error("--corr-every must be >= 1")

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU (the library has no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        return 2

    # the CPU legs run first, before anything touches the GPU (their worker
    # processes start from a clean parent)
    study = args.precision_study > 0 or args.learned_study > 0 or args.jet_study > 0 or args.production_run > 0
    cpu = None
    variant_rates = {}
    if not args.no_cpu_baseline and not study:
        cpu = cpu_baseline(args.cpu_les_steps, args.cpu_dns_steps, args.cpu_all_steps)
        variant_rates = variant_oracle_rates()

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
    if args.learned_study > 0:
        return learned_study(args, dev, stream)
    if args.production_run > 0:
        return production_run(args, dev, stream)
    if args.jet_study > 0:
        return jet_study(args, dev, stream)

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
        # every diag_every steps and at the end of the timed window, so a
        # window shorter than diag_every still contains the diagnostics
        if done % args.diag_every == 0 or done == K:
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
        "kernel": "k_fused_dns_pair<float, float, true, 5> (4096^2 DNS sweep)",
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

    roofline_plain = None
    if args.les4096_steps > 0:
        del les
        # 4096^2 LES (Delta = 4) in every closure variant and schedule, each
        # timed over the same steps from the same state; the end states are
        # compared with the synchronous fused run (relative L2 of m and of
        # B - mean B), beside the closure's own effect (sync LES vs Delta = 0).
        # values per update: fused 19 + 19; in place synchronous 19 + 4 then
        # 19 + 4 + 19; in place lagged 19 + 4 + 19 + 4.
        variants = [
            ("les4096", "fused", {}, 38, "k_fused_les_f<float> (plain closure, Delta=4)"),
            ("les4096_full", "fused", dict(closure="full"), 38, "k_fused_les_f<float, ..., full> (density-gradient terms)"),
            ("les4096_local_iso9", "fused", dict(grad_stencil="local_iso9"), 38,
             "k_fused_les_f<float, LOCAL_ISO9> (gradients from non-equilibrium moments)"),
            ("les4096_aa", "aa", {}, 65, "k_aa_moments + k_aa_les (in place, synchronous)"),
            ("les4096_aa_lagged", "aa_lagged", {}, 46, "k_aa_les_lagged (in place, lagged gradients)"),
            # D2Q9 vector distribution (27 populations): compared with the D2Q5 run
            ("les4096_d2q9", "fused", dict(mag_lattice="d2q9"), 54, "k_fused_les_f<float, ..., QG=9> (D2Q9 g)"),
            ("dns4096_d2q9", "fused", dict(mag_lattice="d2q9", delta=0.0), 54,
             "k_fused_dns_pair<float, QG=9> (D2Q9 g, closure off)"),
        ]
        nsteps = 20 + args.les4096_steps

        def field_rel(a, b):
            da, db = a[1:3] - b[1:3], b[1:3]
            bm = b[3:5].mean(dim=(1, 2), keepdim=True)
            return {"m": float(da.norm() / db.norm()), "B": float((a[3:5] - b[3:5]).norm() / (b[3:5] - bm).norm())}

        sd = Sim(nx=DNS_N, ny=DNS_N, nu=NU, eta=ETA, delta=0.0, dtype="fp32", schedule="fused",
                 b_ref=bref, device=dev, stream=stream, **ghost)
        sd.init_kh_jet(seed=0, **KH)
        sd.step(nsteps)
        mom_off = sd.moments()
        del sd
        mom_sync = None
        for key, sched, kw, vals, kname in variants:
            args_v = dict(nx=DNS_N, ny=DNS_N, nu=NU, eta=ETA, delta=LES_DELTA, dtype="fp32", schedule=sched,
                          b_ref=bref, device=dev, stream=stream, **ghost)
            args_v.update(kw)
            sv = Sim(**args_v)
            sv.init_kh_jet(seed=0, **KH)
            sv.step(20)
            a, b = ev(), ev()
            a.record(stream)
            sv.step(args.les4096_steps)
            b.record(stream)
            torch.cuda.synchronize(dev)
            ms = a.elapsed_time(b) / args.les4096_steps
            bw = vals * 4 * dns_lups / (ms * 1e-3) / 1e9
            rec = {"mlups": round(dns_lups / (ms * 1e-3) / 1e6, 1), "avg_step_us": round(ms * 1e3, 2),
                   "bytes_per_lup": vals * 4, "achieved_GBps": round(bw, 1), "frac": round(bw / HBM_PEAK_GBS, 4),
                   "kernel": kname}
            mom = sv.moments()
            if mom_sync is None:
                mom_sync = mom
                rec["closure_effect_vs_delta0"] = {k: float(f"{v:.3e}") for k, v in field_rel(mom, mom_off).items()}
            else:
                ref = mom_off if args_v["delta"] == 0.0 else mom_sync
                name = "rel_l2_vs_d2q5" if "mag_lattice" in kw else "rel_l2_vs_sync_fused"
                rec[name] = {k: float(f"{v:.3e}") for k, v in field_rel(mom, ref).items()}
                del mom
            extra[key] = rec
            if key == "les4096":
                # the plain closure beyond the caches: one k_fused_les_f launch per step
                roofline_plain = {
                    "bound": "hbm",
                    "kernel": "k_fused_les_f<float, 512, 0, true, 0, 5> (4096^2 LES sweep, plain closure)",
                    "achieved": round(bw, 1),
                    "peak": HBM_PEAK_GBS,
                    "unit": "GB/s",
                    "frac": round(bw / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic("fused_les4096_fp32", dns_lups),
                    "algorithmic_bytes_per_launch": BYTES_PER_LUP_FP32 * dns_lups,
                    "avg_launch_us": round(ms * 1e3, 2),
                    "target_frac": 0.70,
                }
            log(f"{key}: {ms * 1e3:.1f} us/step, {bw:.0f} GB/s algorithmic")
            del sv
        del mom_off, mom_sync
        torch.cuda.empty_cache()

    if args.learned_steps > 0:
        # 1024^2 LES with the learned closure (moments -> network correction on
        # the matrix cores -> fused collision), FP32 and BF16 storage.  The
        # weights are an untrained Glorot draw: the work per cell does not
        # depend on them.
        from paper_1705_09807_amd import learned as G
        mlp = G.Mlp(G.glorot_params(0), device=dev, stream=stream)
        mlp.set_norm(shift=[1.0, 0.0, 0.0, KH["B0"], 0.0, 0.0, 0.0],
                     scale=[1e3, 20.0, 20.0, 100.0, 100.0, 1e3, 1e3], out_scale=[1e-6] * 4)
        packed = mlp.pack()
        n_l = LES_N * LES_N
        legs = [("fp32", 1), ("bf16", 1), ("fp16", 1)]
        if args.corr_every > 1:
            legs += [("fp32", args.corr_every), ("fp16", args.corr_every), ("bf16", args.corr_every)]
        for dt, every in legs:
            sl = Sim(nx=LES_N, ny=LES_N, nu=NU, eta=ETA, delta=LES_DELTA, dtype=dt, schedule="fused",
                     b_ref=bref, closure="learned", device=dev, stream=stream, **ghost)
            sl.init_kh_jet(seed=0, **KH)
            sl.set_closure_mlp(packed)
            sl.set_correction_interval(every)
            sl.step(20)
            # a whole number of intervals: each holds exactly one network evaluation
            nsteps = every * -(-args.learned_steps // every)
            a, b = ev(), ev()
            a.record(stream)
            sl.step(nsteps)
            b.record(stream)
            torch.cuda.synchronize(dev)
            ms = a.elapsed_time(b) / nsteps
            # matrix-core work of the network per cell: 63*64 + 64*64 + 64*4 multiply-adds
            flops = 2 * (63 * 64 + 64 * 64 + 64 * 4) * n_l
            key = f"les1024_learned_{dt}" + (f"_every{every}" if every > 1 else "")
            extra[key] = {
                "mlups": round(n_l / (ms * 1e-3) / 1e6, 1), "avg_step_us": round(ms * 1e3, 2),
                "network_tflops_per_step_time": round(flops / every / (ms * 1e-3) / 1e12, 1),
                "fine_equivalent_mlups": round(64 * n_l / (ms * 1e-3) / 1e6, 1),
                # the analytic-closure FP32 LES of the same grid (the headline run's les1024)
                "speed_vs_plain_fp32_les": round(les_ms / ms, 3),
                "correction_every": every, "steps": nsteps,
                "note": "fine-equivalent: a 4x coarser grid (16x fewer cells) and 4x longer steps "
                        "than the 4096^2 DNS it stands for",
                "kernels": ("k_cell_inputs + k_mlp_correct (bf16 MFMA) + k_fused_les_f<..., CORR>" if every == 1
                            else f"k_cell_inputs + k_mlp_correct every {every} steps, "
                                 "k_fused_les_f<..., CORR> every step")}
            log(f"learned les 1024^2 {dt} (network every {every}): {ms * 1e3:.1f} us/step")
            del sl
        # one Adam step of the network on 8192 rows (forward, matrix-core
        # backward, fixed-order reduction, Adam), synthetic seeded rows
        gen = torch.Generator(device=dev).manual_seed(5)
        Xt = torch.randn((1 << 16, 64), device=dev, generator=gen) * 0.5
        Xt[:, 63] = 0.0
        Tt = torch.randn((1 << 16, 4), device=dev, generator=gen)
        mlp.fit_norm(Xt, Tt)
        from paper_1705_09807_amd import training as TR
        TR.train(mlp, Xt, Tt, steps=20, batch=8192)
        torch.cuda.synchronize(dev)
        a, b = ev(), ev()
        a.record(stream)
        TR.train(mlp, Xt, Tt, steps=200, batch=8192)
        b.record(stream)
        torch.cuda.synchronize(dev)
        ms = a.elapsed_time(b) / 200
        # flops per row: forward 2 * (63 * 64 + 64 * 64 + 64 * 4) = 16 768; backward
        # d1 = W2 d2 (2 * 64 * 64) and the three weight gradients (16 768 again)
        tflop = 8192 * (16768 + 2 * 64 * 64 + 16768) / (ms * 1e-3) / 1e12
        extra["mlp_train_step_8192"] = {"avg_step_us": round(ms * 1e3, 1), "rows": 8192,
                                        "tflops_fwd_bwd": round(tflop, 2),
                                        "kernels": "k_mlp_pack + k_mlp_train (matrix cores) + k_mlp_reduce_groups + k_mlp_reduce + k_mlp_adam"}
        log(f"mlp train step (8192 rows): {ms * 1e3:.1f} us")
        del mlp, packed, Xt, Tt

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

    if args.production_steps > 0:
        # 16384^2 jet (268M cells) with the learned closure, nu = eta = 5e-5,
        # B0 = 0.02, BF16 population storage (the production configuration)
        # and FP16 (the 16-bit storage that keeps the growth rate): the step,
        # and with BF16 the radially binned spectra taken every 1000 steps
        # (moments + FP64 FFTs), timed once.
        from paper_1705_09807_amd import learned as G
        n16, b16 = 16384, 0.02
        kh16 = dict(KH, B0=b16)
        lups16 = n16 * n16
        mlp = G.Mlp(G.glorot_params(0), device=dev, stream=stream)
        mlp.set_norm(shift=[1.0, 0.0, 0.0, b16, 0.0, 0.0, 0.0],
                     scale=[1e3, 20.0, 20.0, 100.0, 100.0, 1e3, 1e3], out_scale=[1e-6] * 4)
        packed = mlp.pack()
        legs = [("bf16", 1), ("fp16", 1)]
        if args.corr_every > 1:
            legs += [("bf16", args.corr_every), ("fp16", args.corr_every)]
        for dt, every in legs:
            sp = Sim(nx=n16, ny=n16, nu=5e-5, eta=5e-5, delta=LES_DELTA, dtype=dt, schedule="fused",
                     b_ref=(b16, 0.0), closure="learned", device=dev, stream=stream, **ghost)
            sp.init_kh_jet(seed=0, **kh16)
            sp.set_closure_mlp(packed)
            sp.set_correction_interval(every)
            sp.step(2)
            # a whole number of intervals: each holds exactly one network evaluation
            nsteps = every * -(-args.production_steps // every)
            a, b = ev(), ev()
            a.record(stream)
            sp.step(nsteps)
            b.record(stream)
            torch.cuda.synchronize(dev)
            ms = a.elapsed_time(b) / nsteps
            rec = {"mlups": round(lups16 / (ms * 1e-3) / 1e6, 1), "avg_step_us": round(ms * 1e3, 1),
                   "steps": nsteps, "correction_every": every,
                   "kernels": (f"k_cell_inputs + k_mlp_correct (bf16 MFMA) + k_fused_les_f<{dt}, ..., CORR>"
                               if every == 1 else
                               f"k_cell_inputs + k_mlp_correct every {every} steps, "
                               f"k_fused_les_f<{dt}, ..., CORR> every step")}
            if dt == "bf16" and every == 1:
                mom16 = torch.empty((5, n16, n16), dtype=torch.float64, device=dev)
                sp.moments(mom16)
                G.spectra(mom16, stream=stream)  # first call: the allocator takes the work buffer
                a.record(stream)
                sp.moments(mom16)
                ek, em, _ = G.spectra(mom16, stream=stream)
                b.record(stream)
                torch.cuda.synchronize(dev)
                ms_spec = a.elapsed_time(b)
                d16 = sp.diagnostics()
                rec.update({
                    "spectra_ms": round(ms_spec, 2),
                    "spectra_share_every_1000_steps": round(ms_spec / (1000 * ms), 5),
                    "nonfinite": int(d16["nonfinite"]), "e_kin": d16["e_kin"], "e_mag": d16["e_mag"],
                    # Parseval: the magnetic spectrum sums to the domain mean <|B|^2 / 2>
                    "parseval_em_rel": float(abs(em.sum().item() - d16["e_mag"]) / d16["e_mag"]),
                    "spectra_kernels": "k_moments_out + k_fft_rows_big + k_fft_cols_big + k_bin_cols + "
                                       "k_spectra_final"})
                log(f"production 16384^2 spectra {ms_spec:.1f} ms")
                del mom16, ek, em
            else:
                rec["nonfinite"] = int(sp.diagnostics()["nonfinite"])
            extra[f"les16384_learned_{dt}" + (f"_every{every}" if every > 1 else "")] = rec
            log(f"production 16384^2 learned {dt} (network every {every}): {ms * 1e3:.0f} us/step")
            del sp
            torch.cuda.empty_cache()
        del mlp, packed
        torch.cuda.empty_cache()

    last_dns, last_les = diag_log[-1] if diag_log else ({}, {})
    out = {
        "metric": "MLUPS + % HBM roofline; learned vs plain closure at \u22642% spectrum error",
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
                        "diagnostics every 100 steps and at the end of the timed window",
            "diagnostics_in_timed_window": len(diag_log),
            "grids": [LES_N, DNS_N],
            "delta": [LES_DELTA, 0.0],
            "U0": KH["U0"], "delta_over_L": KH["delta_over_L"], "B0": KH["B0"], "nu": NU, "eta": ETA,
            "mrt_ghost_rates": GHOST,
            "diag_every": args.diag_every,
            "schedule": "fused",
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "roofline_plain_closure": roofline_plain,
        "extra": extra,
        "diagnostics_last": {"dns": {k: last_dns.get(k) for k in ("t", "e_kin", "e_mag", "enstrophy", "j2")},
                             "les": {k: last_les.get(k) for k in ("t", "e_kin", "e_mag", "enstrophy", "j2")}},
        "cpu_baseline": None,
    }
    del dns
    torch.cuda.empty_cache()
    if args.copy_bytes == 0:
        # what this GPU sustains for a plain stream: a device-to-device copy (torch
        # copy_, the runtime's copy kernel) of the bytes one 4096^2 FP32 sweep moves,
        # 1.275 GB read and 1.275 GB written.  Skipped in counter runs, whose
        # calibration copy (--copy-bytes) must be the only large copy.
        nb = 19 * 4 * DNS_N * DNS_N
        ca = torch.empty(nb, dtype=torch.uint8, device=dev)
        cb = torch.empty_like(ca)
        cb.copy_(ca)
        torch.cuda.synchronize(dev)
        e0, e1 = ev(), ev()
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            cb.copy_(ca)
        e1.record(stream)
        torch.cuda.synchronize(dev)
        ms = e0.elapsed_time(e1) / reps
        gbps = 2 * nb / (ms * 1e-3) / 1e9
        extra["copy_d2d_4096sq_fp32_bytes"] = {
            "avg_us": round(ms * 1e3, 1), "GBps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBS, 4),
            "note": "device-to-device copy of 1.275 GB (torch copy_): the bytes of one 4096^2 FP32 sweep"}
        log(f"copy of {nb / 1e9:.3f} GB: {ms * 1e3:.1f} us, {gbps:.0f} GB/s")
        del ca, cb
        torch.cuda.empty_cache()
    if args.copy_bytes > 0:
        a = torch.empty(args.copy_bytes, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize(dev)
        del a, b
        torch.cuda.empty_cache()
    if cpu is not None:
        out["cpu_baseline"] = cpu
        # the oracle beside each variant leg (its own mode, a 512^2 sample)
        for key, rec in variant_rates.items():
            for k, v in out["extra"].items():
                if k == key or (key == "les1024_learned" and k.startswith(key)):
                    v.update(rec)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
