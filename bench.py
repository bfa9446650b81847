#!/usr/bin/env python3
"""Benchmark of the FP64 FLI phase-space scan and its surrogate-assisted form
on one MI355X.

Default workload (surrogate4096): the surrogate-assisted scan of the
4096 x 4096 (r0, theta) grid -- r0 in [10, 40], spin polar angle theta in
[0, pi] (theta1 = pi/2, theta2 = theta), beta = 1, chi = 1, all Hamiltonian
terms on, RK4 with h = 1 to t = 1e5, the six-integral correction after every
step, FLI threshold 5.8.  The network (7-256-256-256-2, BF16 MFMA) is trained
on the FP64 scan of the 10^6-orbit uneven batch (untimed setup); one benchmark
step is one whole assisted scan of the 16.8 M points (audit integration,
refinement, inference, gate, fallback integration, merge).  value =
grid-pts/s of the assisted scan; plain_* fields give the plain FP64 scan of
the same grid (rate measured on a seeded 65,536-point sample) and the label
agreement between the two.

Other workloads (--workload): grid64 (64 x 64, plain fused scan), grid314,
fig7 (balanced schedule), batch1M (persistent work-stealing batch), single,
fig6, table2, orbit3, gw.  value there = orbit-steps per second (an orbit-step
advances one orbit and its shadow by h, with both corrections and the FLI
update).

roofline: the dominant kernel (the FP64 scan) against the FP64 vector peak,
with the algorithmic work per orbit-step ALG_FLOPS_PER_ORBIT_STEP; hardware
FP64 operations per orbit-step from rocprofv3 counters are reported beside
it while the kernel sources are unchanged.  cpu_baseline: the oracle as it
is, timed on this host on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 orbit-steps/s + scan grid-pts/s (surrogate vs plain, ≥99% FLI label agree)"
FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X: 256 CU x 128 FP64 flop/clk x 2.4 GHz

# Algorithmic FP64 work of one orbit-step with RK4 and the six-integral
# correction (two sweeps), the scope's per-unit figure: about 2 x (2.0k for
# the RK4 step + 0.6k for the correction) + 40 for the separation.  The
# oracle's counting scalar gives 7.7k: it evaluates H and its gradient
# separately, and H again with dH/dp in every momentum-scaling iteration.
# The kernel executes about 5.0k (FP64 instruction counters, FMA = 2).  The
# oracle's count is reported beside the roofline as a secondary figure.
ALG_FLOPS_PER_ORBIT_STEP = 5200.0
KERNEL_SOURCES = ["paper_1802_00147_amd/csrc/pn_kernels.hip", "paper_1802_00147_amd/csrc/pn_device.h"]

# HBM bytes from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (KiB per dispatch,
# scaled by a 1 GiB device copy: FETCH_SIZE x 1.9999, WRITE_SIZE x 1.0),
# valid only for the kernel sources whose hash is recorded with them.
# surrogate4096: the eight k_wrap_scan launches of one assisted scan, 226.4 MB
# read + 180.1 MB written, 50.8 MB per launch; fig7: the three launches of
# the balanced scan, 81.3 MB read + 81.2 MB written, 54.2 MB per launch.
TRAFFIC = dict(sources_sha256="a0a398ce521ad1cbb5af85f3f6c8a6f8a0e6b93ce527798f7dad9423e4a89349",
               bytes_per_launch={"surrogate4096": 406514885 / 8, "fig7": 162541823 / 3})


# Table 3 of the paper: wall time of its GPU and CPU scans (seconds).
PAPER_TABLE3 = {"fig6_th1_1.571": (75.0, 1020.0), "fig7": (2213.0, 25000.0)}


# FP64 operations per orbit-step that the scan kernels execute, from
# rocprofv3 counters (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 x 64 lanes, FMA
# counted twice, over the launch's orbit-steps), valid only for the kernel
# sources whose hash is recorded with them.
HW_FLOPS = dict(sources_sha256="a0a398ce521ad1cbb5af85f3f6c8a6f8a0e6b93ce527798f7dad9423e4a89349",
                per_orbit_step={("k_wrap_scan", "surrogate4096"): 4575.8, ("k_wrap_scan", "grid314"): 4552.4,
                                ("k_wrap_scan", "fig7"): 4598.3, ("k_batch_scan", "batch1M"): 4582.4,
                                ("k_fli_scan", "grid64"): 4550.4})


def hardware_flops(kernel, workload):
    """Hardware FP64 flops per orbit-step of `kernel` on `workload`, from the
    counters recorded above (None when the sources changed or none were
    taken)."""
    if HW_FLOPS["sources_sha256"] != sources_sha256():
        return None
    return HW_FLOPS["per_orbit_step"].get((kernel, workload))


def sources_sha256():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def make_workload(name):
    from paper_1802_00147_amd import workloads as W
    if name == "grid64":
        return W.grid64()
    if name == "grid314":
        return W.grid314()
    if name == "batch1M":
        return W.batch()
    if name == "fig7":
        return W.fig7()
    if name == "single":
        return W.single()
    if name == "fig6":
        return W.fig6()
    raise SystemExit(f"unknown workload {name}")


def describe(wl):
    if wl.name == "single":
        return {"workload": f"single: one orbit and its shadow (d0 = 1e-8), r0=20, p0 from seed 1, beta=1, chi=1, "
                            f"isotropic spins (seed 1), t={wl.t_end:g}, RK4 h=1, six-integral correction, QM on",
                "orbits": 1, "t_end": wl.t_end, "orbit_steps_scheduled": wl.steps()}
    if wl.shape is None:
        return {"workload": f"{wl.name}: {wl.n} orbits, per-orbit beta in [0.1,1], chi in [0,1], isotropic "
                            "spins, r0 in [8,60], t_end log-uniform in [1e3,1e6]; persistent work-stealing "
                            "scan, autotuned; RK4 h=1, six-integral correction, QM on",
                "orbits": wl.n, "orbit_steps_scheduled": wl.steps()}
    if wl.name.startswith("fig6"):
        return {"workload": "fig6: the paper's theta2 line, 314 orbits, theta2 = 0.01k, theta1 = pi/2, "
                            f"(beta, r0, p_y) = (1/3, 5.65, 0.765) as printed (unbound states removed at t = 0), "
                            f"chi=1, QM on, t={wl.t_end:g}, RK4 h=1, six-integral correction, threshold 5.8",
                "orbits": wl.n, "t_end": wl.t_end, "orbit_steps_scheduled": wl.steps()}
    if wl.name == "fig7":
        return {"workload": "fig7: the paper's 314x314 (theta1, theta2) spin-angle plane, theta_i = 0.01k, "
                            f"r0=10.14, p_y=0.365, beta=1, chi=1, QM on, t={wl.t_end:g}, RK4 h=1, "
                            "six-integral correction, threshold 5.8",
                "orbits": wl.n, "t_end": wl.t_end, "orbit_steps_scheduled": wl.steps()}
    return {"workload": f"{wl.name}: {wl.shape[0]}x{wl.shape[1]} FLI scan, t={wl.t_end:g}, RK4 h=1, "
                        f"six-integral correction, beta={wl.beta:g}, chi={wl.chi1:g}, QM "
                        f"{'on' if wl.model.get('quad_mono', 1) else 'off'}",
            "orbits": wl.n, "t_end": wl.t_end, "orbit_steps_scheduled": wl.steps()}


def cpu_baseline(wl, sample, flop_sample_steps=2000):
    """The oracle on a bounded sample of the workload: timing on this host's
    cores, and the oracle's own flops per orbit-step (counting scalar)."""
    import oracle as O
    from paper_1802_00147_amd import workloads as W
    idx = W.strided_sample(wl.n, sample, seed=11)
    # Threads that can work: the host's cores (at most 16, the CPU share of
    # one GPU on a shared host), and no more than the sample has orbits.
    cores = max(1, min(os.cpu_count() or 1, 16, len(idx)))
    sub = wl.subset(idx)
    y0 = O.init_state(sub.r0, sub.p0, sub.th1, sub.ph1, sub.th2, sub.ph2, sub.beta, sub.chi1, sub.chi2,
                      model=wl.model)
    t0 = time.perf_counter()
    res = O.fli_scan(y0, sub.t_end, sub.beta, sub.chi1, sub.chi2, model=wl.model, nthreads=cores)
    dt = time.perf_counter() - t0
    steps = int(res["steps"].sum())
    flops = []
    pick = (lambda v, k: v[k] if isinstance(v, np.ndarray) else v)
    # Flops per orbit-step from up to 8 sample orbits that take steps (a state
    # removed at t = 0 has none to count).
    for k in [k for k in range(len(idx)) if res["steps"][k] > 0][:8]:
        c = O.count_flops(y0[k], float(flop_sample_steps), pick(sub.beta, k), pick(sub.chi1, k),
                          pick(sub.chi2, k), model=wl.model)
        flops.append(c["run_total"] / c["steps"])
    tdesc = f"full t={wl.t_end:g}" if wl.shape is not None else "full per-orbit t_end"
    rate = steps / dt
    return dict(value=rate, unit="orbit-steps/s", cores=cores, kind="oracle",
                sample=f"{len(idx)} seeded orbits of {wl.name}, {tdesc} "
                       f"({steps} orbit-steps, {dt:.1f} s wall on {cores} threads)",
                per_core=rate / cores, nproc=os.cpu_count(), cpu_model=cpu_model(),
                labels=res["label"], oracle_flops_per_orbit_step=float(np.mean(flops)))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def gw_bench(args, dev):
    """Gravitational-wave polarisations (eq. 14) of recorded trajectories: the
    4,096 grid64 orbits integrated 2,000 steps (RK4, six-integral correction)
    with every state recorded (untimed setup), then one benchmark step = one
    pn_gw_polarizations launch over all 8.19e6 samples (face-on observer).
    Algorithmic bytes per sample: 96 read + 16 written."""
    import torch
    from paper_1802_00147_amd import pn, workloads as W

    wl = W.grid64()
    cols = {k: torch.as_tensor(getattr(wl, k), device=dev) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")}
    y = pn.init_state(cols["r0"], cols["p0"], cols["th1"], cols["ph1"], cols["th2"], cols["ph2"], 1.0, 1.0, 1.0)
    rows = 2000
    traj = pn.trajectory(y, 1.0, 1.0, 1.0, rows, 1, correction=dict(mode="six"))
    torch.cuda.synchronize()
    samples = rows * wl.n
    stream = torch.cuda.current_stream(dev)
    for _ in range(max(args.warmup, 1)):
        pn.gw_polarizations(traj, 1.0, 1.0, 1.0, [0, 0, 1], [1, 0, 0], dist=1.0)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        hp, hx = pn.gw_polarizations(traj, 1.0, 1.0, 1.0, [0, 0, 1], [1, 0, 0], dist=1.0)
        b.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    nbytes = samples * (96 + 16)
    achieved = nbytes / (kernel_ms * 1e-3) / 1e9
    line = dict(metric="GW polarisation samples/s (eq. 14, quadrupole field of recorded trajectories)",
                value=samples * args.steps / elapsed, unit="samples/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=1e3 * elapsed / args.steps, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
                config={"workload": f"gw: grid64 orbits (4096), {rows} recorded steps each, RK4 h=1, six-integral "
                                    "correction; h_plus/h_cross for N=z, p=x", "samples": samples},
                finite_fraction=float(torch.isfinite(hp).float().mean().item()),
                roofline=dict(bound="hbm", achieved=achieved, peak=8000.0, unit="GB/s", frac=achieved / 8000.0,
                              traffic=None, kernel="k_gw", kernel_ms=kernel_ms, bytes_per_sample=112))
    print(json.dumps(line), flush=True)


def _single_orbit_flops(wl, model, integrator, correction):
    """Algorithmic flops of one corrected step of one trajectory (oracle
    counting scalar)."""
    import oracle as O
    y0 = O.init_state(wl.r0, wl.p0, wl.th1, wl.ph1, wl.th2, wl.ph2, wl.beta, wl.chi1, wl.chi2, model=model)
    c = O.count_flops(y0[0], 10.0, wl.beta, wl.chi1, wl.chi2, integrator=integrator, correction=correction)
    return c["rk_step"] + c["correction"]


def table2_bench(args, dev):
    """The paper's Table 2 protocol (Sec. 3B): each of the four test orbits
    (Cases I-II, orbits 1-2) integrated to t = 1e5 with RK5 (h = 1), corrected
    by the dual scaling at eps = 1e-10 (the paper's correction) and
    uncorrected; energy error max |H - E0| / |E0| over checkpoints every 1e4,
    GPU elapsed time (one orbit, one lane: a latency-bound launch) against the
    oracle on one host core.  One benchmark step = the four corrected runs."""
    import torch
    import oracle as O
    from paper_1802_00147_amd import pn, workloads as W

    integ = dict(method=1, h=1.0)
    dual = dict(mode=3, tol=1e-10)
    nchunk, chunk = 10, 10000
    stream = torch.cuda.current_stream(dev)
    rows, gpu_ms = [], 0.0
    for name in ("I-1", "I-2", "II-1", "II-2"):
        wl = W.paper_orbit(name)
        args_p = (wl.beta, wl.chi1, wl.chi2)
        y0 = pn.init_state(*[torch.as_tensor(getattr(wl, k), device=dev) for k in ("r0", "p0", "th1", "ph1", "th2",
                                                                                     "ph2")], *args_p)
        H0, J0 = pn.invariants(y0, *args_p)
        ref = torch.cat([H0.reshape(1, 1), J0.reshape(3, 1)]).contiguous()
        e0 = float(H0[0])
        res = {}
        for label, corr in (("corrected", dual), ("uncorrected", None)):
            y = y0.clone()
            err, ms = 0.0, 0.0
            for _ in range(nchunk):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                pn.step(y, *args_p, chunk, integrator=integ, correction=corr, ref=ref)
                b.record(stream)
                H, _ = pn.invariants(y, *args_p)
                torch.cuda.synchronize()
                ms += a.elapsed_time(b)
                err = max(err, abs(float(H[0]) - e0) / abs(e0))
            res[label] = (err, ms)
        gpu_ms += res["corrected"][1]
        # The oracle's corrected run, one host core.
        yo = O.init_state(wl.r0, wl.p0, wl.th1, wl.ph1, wl.th2, wl.ph2, *args_p)
        Ho, Jo = O.invariants(yo, *args_p)
        t0 = time.perf_counter()
        yo = O.step(yo, *args_p, nchunk * chunk, integrator=integ, correction=dual)
        cpu_s = time.perf_counter() - t0
        rows.append(dict(orbit=name, dE_corrected=res["corrected"][0], dE_uncorrected=res["uncorrected"][0],
                         gpu_s=res["corrected"][1] * 1e-3, gpu_s_uncorrected=res["uncorrected"][1] * 1e-3,
                         oracle_s=cpu_s, us_per_step=1e3 * res["corrected"][1] / (nchunk * chunk)))
    steps = 4 * nchunk * chunk
    fps = float(np.mean([_single_orbit_flops(W.paper_orbit(r["orbit"]), None, integ, dual) for r in rows]))
    achieved = fps * steps / (gpu_ms * 1e-3) / 1e12
    cpu_total = sum(r["oracle_s"] for r in rows)
    line = dict(metric="Table 2 protocol: corrected RK5 steps/s of one test orbit and its energy error",
                value=steps / (gpu_ms * 1e-3), unit="steps/s", n_gpus=1, steps=1, warmup=0,
                ms_per_step=gpu_ms, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
                data="synthetic",
                config={"workload": "table2: the paper's Case I/II test orbits 1-2 (Sec. 3B), RK5 h=1 to t=1e5, "
                                    "dual scaling eps=1e-10 (and uncorrected), energy error over checkpoints "
                                    "every 1e4", "orbits": 4, "t_end": 1e5},
                rows=rows,
                latency=dict(us_per_step=1e3 * gpu_ms / steps, wavefronts=1, simd_fraction=1.0 / 1024),
                cpu_baseline=dict(value=steps / cpu_total, unit="steps/s", cores=1, kind="oracle",
                                  sample="the same four corrected runs on one host thread", cpu_model=cpu_model()),
                roofline=dict(bound="alu", achieved=achieved, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                              frac=achieved / FP64_VECTOR_PEAK_TFLOPS, traffic=None, kernel="k_step<RK5,DUAL>",
                              kernel_ms=gpu_ms / 4, flops_per_step=fps))
    print(json.dumps(line), flush=True)


def orbit3_bench(args, dev):
    """The paper's dissipative orbit 3 (Sec. 3B, Fig. 5): the full Hamiltonian
    with the 2.5PN reaction, RK5 (h = 1) corrected by the dual scaling
    (eps = 1e-10) against references that follow the integral-invariant
    relation, integrated in chunks (at most 2e4 steps) until r < 6 (or t = 1e6).
    Reports the inspiral time, the energy error against the advancing
    reference and the GPU time per step (one lane, latency-bound) beside the
    oracle running the same inspiral on one host core."""
    import torch
    import oracle as O
    from paper_1802_00147_amd import pn, workloads as W

    model = dict(rad_reaction=1)
    integ = dict(method=1, h=1.0)
    dual = dict(mode=3, tol=1e-10)
    chunk, r_stop, t_max = 20000, 6.0, 1_000_000
    wl = W.paper_orbit("orbit3")
    args_p = (wl.beta, wl.chi1, wl.chi2)
    y = pn.init_state(*[torch.as_tensor(getattr(wl, k), device=dev) for k in ("r0", "p0", "th1", "ph1", "th2",
                                                                               "ph2")], *args_p)
    H0, J0 = pn.invariants(y, *args_p, model=model)
    ref = torch.cat([H0.reshape(1, 1), J0.reshape(3, 1)]).contiguous()
    stream = torch.cuda.current_stream(dev)
    t, ms, err, r = 0, 0.0, 0.0, float(wl.r0[0])
    chunks = []
    while t < t_max:
        # Chunks of 5% of the remaining quadrupole inspiral time at the current
        # separation, (5/256) r^4 / eta, so that the run stops at r_stop and
        # not in the plunge that follows.
        eta = wl.beta / (1.0 + wl.beta) ** 2
        n = int(min(chunk, max(20, 0.05 * (5.0 / 256.0) * r ** 4 / eta)))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pn.step(y, *args_p, n, model=model, integrator=integ, correction=dual, ref=ref)
        b.record(stream)
        H, _ = pn.invariants(y, *args_p, model=model)
        torch.cuda.synchronize()
        ms += a.elapsed_time(b)
        t += n
        chunks.append(n)
        err = max(err, abs(float(H[0]) - float(ref[0, 0])) / abs(float(ref[0, 0])))
        r = float(torch.linalg.norm(y[0:3, 0]))
        if not np.isfinite(r) or r < r_stop:
            break
    # The oracle on the same inspiral (the same chunks), one host core.
    yo = O.init_state(wl.r0, wl.p0, wl.th1, wl.ph1, wl.th2, wl.ph2, *args_p)
    Ho, Jo = O.invariants(yo, *args_p, model=model)
    refo = np.column_stack([Ho, Jo])
    t0 = time.perf_counter()
    for n in chunks:
        yo, refo = O.step(yo, *args_p, n, model=model, integrator=integ, correction=dual, ref=refo,
                          return_ref=True)
    cpu_s = time.perf_counter() - t0
    ro = float(np.linalg.norm(yo[0, 0:3]))
    fps = _single_orbit_flops(wl, None, integ, dual)
    achieved = fps * t / (ms * 1e-3) / 1e12
    line = dict(metric="Dissipative orbit 3: corrected RK5 steps/s with the 2.5PN reaction",
                value=t / (ms * 1e-3), unit="steps/s", n_gpus=1, steps=1, warmup=0, ms_per_step=ms,
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
                config={"workload": "orbit3: the paper's dissipative test orbit (beta=1, r=50, p_y=0.140, S1 at "
                                    "45 deg, S2 at 30 deg, chi=(1, 0.85)), full Hamiltonian + 2.5PN reaction, "
                                    "RK5 h=1, dual scaling eps=1e-10 against integral-invariant references, "
                                    f"until r < {r_stop:g} (chunks of 5% of the remaining inspiral time)", "orbits": 1},
                t_inspiral=t, r_final=r, r_final_oracle=ro, energy_error_vs_reference=err,
                energy_radiated_fraction=float(ref[0, 0]) / float(H0[0]) - 1.0,
                energy_ref_oracle_rel_diff=abs(float(ref[0, 0]) - float(refo[0, 0])) / abs(float(refo[0, 0])),
                latency=dict(us_per_step=1e3 * ms / t, wavefronts=1, simd_fraction=1.0 / 1024),
                cpu_baseline=dict(value=t / cpu_s, unit="steps/s", cores=1, kind="oracle",
                                  sample="the same inspiral on one host thread", cpu_model=cpu_model()),
                roofline=dict(bound="alu", achieved=achieved, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                              frac=achieved / FP64_VECTOR_PEAK_TFLOPS, traffic=None,
                              kernel="k_step<RK5,DUAL,reaction>", kernel_ms=ms, flops_per_step_conservative=fps))
    print(json.dumps(line), flush=True)


def surrogate_bench(args, dev):
    """Surrogate-assisted scan of the 4096 x 4096 (r0, theta) grid at t = 1e5
    against the plain FP64 scan.  The network is trained on the FP64 scan of
    the 10^6-orbit uneven batch (untimed setup, reported); one benchmark step
    is the whole assisted scan: features, inference, gate, integration of the
    uncertain and audited points, merge.  The plain scan's rate and the label
    agreement come from a seeded sample of grid points integrated by the plain
    kernel."""
    import torch
    from paper_1802_00147_amd import pn, surrogate as S, workloads as W

    t0 = time.perf_counter()
    tr = W.batch()
    tcols = [torch.as_tensor(getattr(tr, k), device=dev) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")]
    tb, tc1, tc2, tt = (torch.as_tensor(getattr(tr, k), device=dev) for k in ("beta", "chi1", "chi2", "t_end"))
    y0 = pn.init_state(*tcols, tb, tc1, tc2)
    sc = pn.batch_scan(y0, tt, tb, tc1, tc2, full=False)
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    ts = S.training_set(tr, sc, dev)
    net, hist = S.train(ts, epochs=args.epochs, batch=4096, lr=1e-3, device=dev)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del y0, sc

    grid = W.grid4096()
    base = [t_.clone() for t_ in net.w + net.b + net.wb + net.mw + net.vw + net.mb + net.vb]
    base_step = net.step

    def restore():   # each assisted scan refines the network trained on batch1M afresh
        for dst, src in zip(net.w + net.b + net.wb + net.mw + net.vw + net.mb + net.vb, base):
            dst.copy_(src)
        net.step = base_step

    def one_scan(ws):
        return S.surrogate_scan(net, grid, ts.stats, margin=args.margin, audit=0.01, seed=5,
                                refine_epochs=args.refine, ws=ws)

    ws = None
    for _ in range(args.warmup):
        restore()
        ws = one_scan(ws).ws
    # Timed region: K whole assisted scans, bracketed by device
    # synchronisation; each scan also reports the duration of its FP64 scan
    # launches (events on the launch stream, inside the library call).
    res = None
    scans = []
    restore()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        if k > 0:
            restore()
        res = one_scan(ws)
        ws = res.ws
        scans.append(res.scans)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # The network's own kernel: fused inference over every grid point against
    # its matrix-core roofline (2 x 133,376 multiply-adds per point), and the
    # layer-by-layer path it replaces.  Five untimed launches first: after the
    # host-side gap the chip's clock ramps from about 1.9 to 2.3 GHz over the
    # first few launches, and the roofline is taken at the settled clock, as
    # the FP64 kernels' (which run for seconds) are.
    feat = S.workload_features(grid, ts.stats, dev)
    stream = torch.cuda.current_stream(dev)
    inf = {}
    for name, fn in (("fused", lambda: pn.mlp_infer_fused(net, feat)),
                     ("layered", lambda: pn.mlp_infer(net, feat, chunk=1 << 20))):
        for _ in range(5):
            fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        inf[name + "_ms"] = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    del feat
    inf_flops = 2.0 * (7 * 256 + 256 * 256 + 256 * 256 + 256 * 2) * grid.n
    inf_achieved = inf_flops / (inf["fused_ms"] * 1e-3) / 1e12

    # Plain scan on a seeded sample of the grid: rate and label agreement.
    # 65,536 orbits fill every SIMD with two wavefronts, as the whole grid
    # (256 times as many, an exact multiple) would.
    idx = W.strided_sample(grid.n, args.plain_sample, seed=17)
    sub = grid.subset(idx)
    scols = [torch.as_tensor(getattr(sub, k), device=dev) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")]
    ys = pn.init_state(*scols, 1.0, 1.0, 1.0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    plain = pn.fli_scan(ys, grid.t_end, 1.0, 1.0, 1.0, full=False)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    plain_steps = int(plain["steps"].sum().item())
    plain_pts_s = len(idx) / (plain_ms * 1e-3)
    got = res.label.cpu().numpy()[idx]
    ref = plain["label"].cpu().numpy()
    agree = float(np.mean(got == ref))
    value = grid.n * args.steps / elapsed
    line = dict(metric=METRIC, value=value, unit="grid-pts/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                ms_per_step=1e3 * elapsed / args.steps, higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f64+bf16", data="synthetic",
                config={"workload": "grid4096 surrogate-assisted FLI scan: 4096x4096 (r0, theta) grid, t=1e5, "
                                    "beta=1, chi=1, QM on, RK4 h=1, six-integral correction; MLP 7-256-256-256-2 "
                                    "(BF16 MFMA, FP32 accumulation) trained on the FP64 scan of batch1M, refined "
                                    "on the integrated 1% SplitMix64 audit of the grid; integration fallback for "
                                    "|logit| < margin",
                        "grid_points": grid.n, "t_end": grid.t_end, "train_epochs": args.epochs,
                        "refine_epochs": args.refine, "margin": args.margin})
    line["plain_grid_pts_per_s"] = plain_pts_s
    line["plain_orbit_steps_per_s"] = plain_steps / (plain_ms * 1e-3)
    line["speedup_vs_plain"] = value / plain_pts_s
    line["label_agreement"] = agree
    line["label_agreement_sample"] = len(idx)
    line["integrated_fraction"] = res.integrated / grid.n
    line["timings_s"] = dict(res.timings, training_data=data_s, training=train_s)
    line["train_loss"] = [round(h, 5) for h in hist]

    # Dominant kernel of the assisted scan: the FP64 scan of the audit and of
    # the uncertain points.  Per launch: the algorithmic work of the
    # orbit-steps it integrated over its average duration, from the scan
    # launches' own events over the timed scans.
    per_kernel = {}
    for sc_k in scans:
        for ph in sc_k:
            if ph["kernel"] is None:
                continue
            d = per_kernel.setdefault(ph["kernel"], dict(ms=0.0, launches=0, orbit_steps=0))
            d["ms"] += ph["ms"]
            d["launches"] += ph["launches"]
            d["orbit_steps"] += ph["orbit_steps"]
    kname, kd = max(per_kernel.items(), key=lambda kv: kv[1]["ms"])
    launch_ms = kd["ms"] / kd["launches"]
    flops_per_launch = ALG_FLOPS_PER_ORBIT_STEP * kd["orbit_steps"] / kd["launches"]
    achieved = flops_per_launch / (launch_ms * 1e-3) / 1e12
    traffic = None
    if TRAFFIC["sources_sha256"] == sources_sha256():
        traffic = TRAFFIC["bytes_per_launch"].get("surrogate4096")
    line["roofline"] = dict(bound="alu", achieved=achieved, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                            frac=achieved / FP64_VECTOR_PEAK_TFLOPS, traffic=traffic,
                            kernel=f"{kname}<RK4,SIX> (audit and fallback integrations of pn_surrogate_scan)",
                            kernel_ms=launch_ms, launches_per_step=kd["launches"] / args.steps,
                            orbit_steps_per_launch=kd["orbit_steps"] / kd["launches"],
                            flops_per_orbit_step=ALG_FLOPS_PER_ORBIT_STEP,
                            orbit_steps_per_s=kd["orbit_steps"] / (kd["ms"] * 1e-3),
                            phases=res.scans)
    hw = hardware_flops(kname, "surrogate4096")
    if hw is not None:
        line["roofline"]["hw_flops_per_orbit_step"] = hw
        line["roofline"]["hw_frac"] = hw * kd["orbit_steps"] / (kd["ms"] * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS
    if kname == "k_wrap_scan":
        line["roofline"]["resources"] = pn.balanced_kernel_resources()
    line["inference_roofline"] = dict(bound="mfma", achieved=inf_achieved, peak=2500.0, unit="TFLOP/s",
                                      frac=inf_achieved / 2500.0, traffic=None, kernel="k_mlp_infer",
                                      kernel_ms=inf["fused_ms"], layered_ms=inf["layered_ms"],
                                      flops_per_point=inf_flops / grid.n)
    plain_tf = ALG_FLOPS_PER_ORBIT_STEP * plain_steps / (plain_ms * 1e-3) / 1e12
    line["plain_roofline"] = dict(bound="alu", achieved=plain_tf, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                                  frac=plain_tf / FP64_VECTOR_PEAK_TFLOPS,
                                  kernel="k_fli_scan<RK4,SIX> (plain scan of the 65,536-point sample)",
                                  kernel_ms=plain_ms)
    if not args.no_cpu_baseline:
        # The oracle's plain scan of seeded points of the same grid, on this
        # host's cores, in grid points per second.
        cb = cpu_baseline(grid, args.cpu_sample)
        cb.pop("labels")
        line["roofline"]["oracle_flops_per_orbit_step"] = cb.pop("oracle_flops_per_orbit_step")
        cb["value"] = cb["value"] / grid.t_end   # orbit-steps/s -> grid-pts/s (1e5 steps per point)
        cb["per_core"] = cb["per_core"] / grid.t_end
        cb["unit"] = "grid-pts/s"
        cb["extrapolated_full_s"] = grid.n / cb["value"]   # plain scan of the whole grid, never run
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="surrogate4096")
    ap.add_argument("--cpu-sample", type=int, default=160)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", choices=("auto", "plain"), default="auto",
                    help="equal-length grids: the library's choice (balanced where it predicts it faster) "
                         "or always the plain fused scan")
    ap.add_argument("--epochs", type=int, default=20, help="surrogate workload: training epochs (cosine decay)")
    ap.add_argument("--plain-sample", type=int, default=65536, help="surrogate workload: plain-scan sample")
    ap.add_argument("--refine", type=int, default=40, help="surrogate workload: refinement epochs on the audit")
    ap.add_argument("--margin", type=float, default=0.5, help="surrogate workload: logit margin of the gate")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of this many MiB (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); the scan shards "
              "by orbits with no exchange during integration, one process per GPU on its share of the "
              "orbits.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1802_00147_amd import pn

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "surrogate4096":
        surrogate_bench(args, dev)
        return
    if args.workload == "gw":
        gw_bench(args, dev)
        return
    if args.workload == "table2":
        table2_bench(args, dev)
        return
    if args.workload == "orbit3":
        orbit3_bench(args, dev)
        return
    wl = make_workload(args.workload)
    cols = {k: torch.as_tensor(getattr(wl, k), device=dev) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")}
    n = wl.n
    out = pn.scan_outputs(n, n, dev, full=True)
    stream = torch.cuda.current_stream(dev)
    batched = wl.shape is None and wl.name != "single"
    as_dev = (lambda v: torch.as_tensor(v, device=dev) if isinstance(v, np.ndarray) else v)
    beta, chi1, chi2, t_end = as_dev(wl.beta), as_dev(wl.chi1), as_dev(wl.chi2), as_dev(wl.t_end)
    kernel = "k_fli_scan<RK4,SIX>"
    sched, bws = None, None
    if not batched:
        # Equal-length grids: the balanced schedule where the library predicts
        # it faster than the plain fused scan (full-chip grids whose resident
        # rounds do not divide evenly), else the plain scan.
        sched = pn.balanced_schedule(n, float(wl.t_end))
        if args.schedule == "plain":
            sched = dict(sched, launches=0)
        if sched["launches"] > 0:
            bws = pn.balanced_workspace(sched["slots"], dev)
            kernel = (f"k_wrap_scan<RK4,SIX> (balanced: {sched['slots']} slots x {sched['slot_len']} steps, "
                      f"{sched['launches']} launches)")
    if batched:
        ws = pn.batch_workspace(n, dev)
        y = pn.init_state(cols["r0"], cols["p0"], cols["th1"], cols["ph1"], cols["th2"], cols["ph2"],
                          beta, chi1, chi2, model=wl.model)
        tuning, _ = pn.autotune_batch(y, t_end, beta, chi1, chi2, model=wl.model, step_scale=0.01, ws=ws,
                                      out=out)
        kernel = f"k_batch_scan<RK4,SIX> {tuning}"

    def one_step(ev=None):
        y = pn.init_state(cols["r0"], cols["p0"], cols["th1"], cols["ph1"], cols["th2"], cols["ph2"],
                          beta, chi1, chi2, model=wl.model)
        if ev is not None:
            ev[0].record(stream)
        if batched:
            pn.batch_scan(y, t_end, beta, chi1, chi2, model=wl.model, out=out, ws=ws)
        else:
            if bws is not None:
                pn.fli_scan_balanced(y, float(t_end), beta, chi1, chi2, model=wl.model, out=out, ws=bws)
            else:
                pn.fli_scan(y, float(t_end), beta, chi1, chi2, model=wl.model, out=out)
        if ev is not None:
            ev[1].record(stream)
        return y

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step(events[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))

    # Orbit-steps actually integrated: an orbit removed early (unbound start,
    # merger, escape) stops counting where it stopped.
    orbit_steps = int(out["steps"].sum())
    value = orbit_steps * args.steps / elapsed
    labels = out["label"].cpu().numpy()
    status = out["status"].cpu().numpy()

    line = dict(metric=METRIC, value=value, unit="orbit-steps/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=1e3 * elapsed / args.steps, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f64", data="synthetic", config=describe(wl))
    line["config"]["orbit_steps"] = orbit_steps
    line["grid_pts_per_s"] = n * args.steps / elapsed
    line["chaotic_fraction"] = float(np.mean(labels == 1))
    line["invalid_orbits"] = int(np.sum((status & 0xFF) != 0))
    simds = 4 * torch.cuda.get_device_properties(dev).multi_processor_count
    balanced = sched is not None and sched["launches"] > 0
    if not batched:
        # Latency view: time per step of the time loop and the share of the
        # chip's SIMDs the trajectories can occupy.
        waves = (sched["slots"] + 31) // 32 if balanced else (2 * n + 63) // 64
        line["latency"] = dict(us_per_step=1e3 * kernel_ms / float(np.max(wl.t_end)), wavefronts=waves,
                               simd_fraction=min(1.0, waves / simds))
        if balanced:
            line["config"]["schedule"] = dict(kind="balanced", **sched)
        else:
            line["config"]["schedule"] = dict(kind="plain")

    if wl.name in PAPER_TABLE3:
        # The paper's own wall times for the same scan (its Table 3, other
        # hardware and integrator): context beside this run's time, never the
        # target.
        gpu_s, cpu_s = PAPER_TABLE3[wl.name]
        line["paper_context"] = dict(table3_gpu_s=gpu_s, table3_cpu_core_s=cpu_s, this_run_s=1e-3 * kernel_ms,
                                     note="GT 650M (RK5) and one i5-3230M core in the paper; context only")
    oracle_fpos = None
    if not args.no_cpu_baseline:
        cb = cpu_baseline(wl, args.cpu_sample)
        oracle_fpos = cb.pop("oracle_flops_per_orbit_step")
        cb.pop("labels")
        # The whole workload on the same host threads, extrapolated from the
        # sample's rate (never run).
        cb["extrapolated_full_s"] = orbit_steps / cb["value"]
        line["cpu_baseline"] = cb
    achieved = ALG_FLOPS_PER_ORBIT_STEP * orbit_steps / (kernel_ms * 1e-3) / 1e12
    traffic = None
    if TRAFFIC["sources_sha256"] == sources_sha256():
        traffic = TRAFFIC["bytes_per_launch"].get(wl.name if args.schedule == "auto" else wl.name + "/plain")
    line["roofline"] = dict(bound="alu", achieved=achieved, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                            frac=achieved / FP64_VECTOR_PEAK_TFLOPS, traffic=traffic,
                            kernel=kernel, kernel_ms=kernel_ms,
                            flops_per_orbit_step=ALG_FLOPS_PER_ORBIT_STEP,
                            oracle_flops_per_orbit_step=oracle_fpos)
    hw = hardware_flops(kernel.split("<")[0], wl.name)
    if hw is not None:
        line["roofline"]["hw_flops_per_orbit_step"] = hw
        line["roofline"]["hw_frac"] = (hw * orbit_steps / (kernel_ms * 1e-3) / 1e12 /
                                       FP64_VECTOR_PEAK_TFLOPS)
    if not batched:
        # Registers, spills and occupancy of the scan kernel as the
        # runtime reports them, and the wavefronts per SIMD the launch
        # actually keeps resident.
        if balanced:
            res = pn.balanced_kernel_resources()
            res["achieved_waves_per_simd"] = min(float(res["waves_per_simd"]),
                                                 ((sched["slots"] + 31) // 32) / simds)
        else:
            res = pn.scan_kernel_resources()
            res["achieved_waves_per_simd"] = min(float(res["waves_per_simd"]), ((2 * n + 63) // 64) / simds)
        line["roofline"]["resources"] = res
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
