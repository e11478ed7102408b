"""Benchmark of the fused N-phase LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
    python bench.py --only spheres_fp64|spheres_fp32|bands_fp32|bands_fp64|rti_fp64|rti_fp32|adjoint_step
                    [--steps K] [--warmup W]

Workload: 512 x 512 periodic D2Q9, N = 4 phases, 40 seeded non-overlapping discs radii
U[10, 30] in an ambient phase, densities 1:2:3:4, sigma_pq U[0.005, 0.02], Model B
(also timed: Model A n = 1, and the FP32 deviation-storage form).  One step = one fused
time step of every phase-field set and the flow set over the whole grid (one kernel
launch), inputs resident in HBM.  Prints ONE JSON line.

value = FP64 Model B MLUPS (node updates per second / 1e6); the FP32 form, Model A and
the oracle on the host (cpu_baseline) are reported beside it, and (unless --no-extra)
the 256^3 D3Q19 N = 4 drops (FP64, FP32), the 2048^2 N = 5 layered bands (FP32, FP64), the
walled ternary Rayleigh-Taylor instability of Sec. 4.4 on 256 x 1024 (FP64, FP32; timing
and the interface locations at T = 1, 2, 3), the wall time of a differentiable 256^2
run (forward with checkpoints, adjoint backward) and the adjoint step alone (HIP events).
`--only NAME` times one of those other workloads alone (for profiling) and prints its
record instead of the line.  roofline: the step kernel is HBM-bound (no dense contraction); achieved = algorithmic bytes per launch
(every persisted value read once and written once) / mean launch time measured with
HIP events on the stream the library launches on.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak, GB/s


def algorithmic_bytes_per_node(d, Q, NS, tsize):
    """Population form of the method's state per node: f (NS*Q), g without the rest slot
    (Q-1), phi^{t-1} (NS), u^{t-1} (d), m_phi^{t-1} (d); each read once and written once.
    This is the per-unit figure the roofline is quoted on."""
    return 2 * (NS * Q + (Q - 1) + NS + 2 * d) * tsize


def algorithmic_bytes_per_node_moment_form(d, Q, NS, tsize):
    """The state the library keeps: each evolved set in moment form (phi, A, D: 1 + 2d
    values; FP32 also the rounding residual of phi; phi doubles as phi^{t-1}), g without
    the rest slot (Q-1), u^{t-1} (d), m_phi^{t-1} (d); each read once and written once.
    The lower floor the moment form reaches, quoted beside the roofline."""
    per_set = 1 + 2 * d + (1 if tsize == 4 else 0)
    return 2 * (NS * per_set + (Q - 1) + 2 * d) * tsize


# sources of the timed step kernels (the adjoint and the host code do not enter a step)
STEP_SOURCES = ("lattice.hpp", "step_kernel.hpp", "step3d_kernel.hpp", "aux_kernels.hpp",
                "dispatch.hpp", "kernels_tu.inc", "kernels_f64_d2q9.hip",
                "kernels_f32_d2q9.hip", "kernels_f64_d3q19.hip", "kernels_f32_d3q19.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_06983_amd", "csrc")
    for fn in STEP_SOURCES:
        h.update(open(os.path.join(csrc, fn), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken with the current kernel sources (else None)."""
    fn = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(fn):
        return None
    try:
        rec = json.load(open(fn))
    except Exception:
        return None
    ent = rec.get(f"{workload}:{precision}")
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def time_gpu(cfg, phi, precision, steps, warmup):
    import torch
    from paper_2306_06983_amd import binding as B
    sim = B.Sim(cfg, precision).init(phi)
    m0 = sim.mass()
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = sim.stream   # the stream the library launches on
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    m1 = sim.mass()
    finite = sim.check()
    phi_out = sim.fields()[0]
    loc = sim.interface_locations(phi_out)   # Sec. 4.4 diagnostics of the final state
    sim.close()
    return dict(ms_total=ms, ms_per_step=ms / steps, wall_s=wall, m0=m0, m1=m1,
                finite=finite, phi=phi_out, locations=loc)


def time_extra(cfg, phi, precision, steps, warmup, d, Q, NS, label):
    """One more workload of the same step: MLUPS and achieved GB/s on the algorithmic
    bytes of the state the library keeps for it (D2Q9: populations; D3Q19: the phase
    field in moment form, with the population-form figure beside it for context)."""
    r = time_gpu(cfg, phi, precision, steps, warmup)
    V = cfg["nx"] * cfg["ny"] * cfg["nz"]
    ts = 8 if precision == "fp64" else 4
    b = algorithmic_bytes_per_node(d, Q, NS, ts)
    mf = algorithmic_bytes_per_node_moment_form(d, Q, NS, ts)
    mlups = V / (r["ms_per_step"] * 1e-3) / 1e6
    gbs = mlups * 1e6 * b / 1e9
    rec = {"workload": label, "precision": precision, "model": cfg["model"],
           "mlups": round(mlups, 1), "ms_per_step": round(r["ms_per_step"], 4),
           "steps_timed": steps, "bytes_per_node_update": b, "achieved_GBs": round(gbs, 1),
           "frac": round(gbs / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic(label, precision), "finite": bool(r["finite"]),
           "moment_form_bytes_per_node_update": mf,
           "moment_form_GBs": round(mlups * 1e6 * mf / 1e9, 1),
           # per phase after warm-up + timed steps: Y_av, Y_min, Y_max (rows / z planes)
           "interface_locations": {"steps": steps + warmup,
                                   "Y_av": [round(float(v), 3) for v in r["locations"][0]],
                                   "Y_min": [int(v) for v in r["locations"][1]],
                                   "Y_max": [int(v) for v in r["locations"][2]]}}
    if d == 3:
        # the per-node moments buffer (phi, j; FP32 residual) written by one pass and read
        # by the next: bytes of this implementation beyond the algorithmic figure
        rec["moments_buffer_bytes_per_node_update"] = 2 * NS * (4 + (1 if ts == 4 else 0)) * ts
    return rec


def rti_diagnostics(precision, model="B", T_marks=(1.0, 2.0, 3.0)):
    """The walled ternary Rayleigh-Taylor run on 256 x 1024 to the given times T (the
    paper's unit t / sqrt(d / (g At))): per phase the interface locations Y_av, Y_min and
    Y_max (C-ABI diagnostics) in the paper's coordinate y / d, y in [-2d, 2d]."""
    from paper_2306_06983_amd import binding as B
    from paper_2306_06983_amd import inputs
    cfg, phi, spt = inputs.ternary_rti(model=model)
    d = cfg["nx"]
    sim = B.Sim(cfg, precision).init(phi)
    m0 = sim.mass()
    out, done = {}, 0
    for T in T_marks:
        n = int(round(T * spt)) - done
        sim.step(n)
        done += n
        av, lo, hi = sim.interface_locations()
        to_y = lambda h: [round((float(v) + 0.5 - 2 * d) / d, 4) for v in h]
        out[f"T={T:g}"] = {"steps": done, "Y_av": to_y(av), "Y_min": to_y(lo), "Y_max": to_y(hi)}
    m1 = sim.mass()
    out["finite"] = bool(sim.check())
    out["mass_drift_rel"] = float(max(abs(m1 - m0) / abs(m0)))
    sim.close()
    return out


def time_adjoint(steps=25, ckpt_every=10):
    """Differentiable run on the 256^2 N = 3 touching discs, loss = L2 misfit of phi(T) to
    a run with sigma_pq scaled by seeded U[0.8, 1.2]: wall time of the forward (with
    checkpoints) and of the backward (segment recompute + hand-written adjoint steps) for
    the FP64 form and for the FP32 form (FP32 forward, FP64 adjoint steps along it), each
    after an untimed warm-up run, and max |dL/dsigma(FP32) - dL/dsigma(FP64)| relative to
    max |dL/dsigma(FP64)|.  25 steps: the horizon at which the FP64 gradient of this
    workload agrees with converged finite differences to 1e-6."""
    import numpy as np
    import torch
    from paper_2306_06983_amd import binding as B
    from paper_2306_06983_amd import inputs
    from paper_2306_06983_amd.autograd import run_differentiable
    cfg, phi = inputs.two_discs(scale=4)
    N = cfg["n_phases"]
    pairs = inputs.sigma_pairs(cfg)
    rng = np.random.default_rng(5)
    tsim = B.Sim(inputs.with_sigma_pairs(cfg, pairs * rng.uniform(0.8, 1.2, size=len(pairs))),
                 "fp64").init(phi)
    tsim.step(steps)
    target = tsim.fields()[0]
    tsim.close()
    out = {"workload": "two_discs_256x256_N3_d2q9_adjoint", "steps": steps,
           "ckpt_every": ckpt_every}
    grads = {}
    for prec in ("fp64", "fp32"):
        for rep in range(2):   # the first run warms up the allocator and the kernels
            phi0 = torch.tensor(phi, dtype=torch.float64, device="cuda:0", requires_grad=True)
            sig = torch.tensor(pairs, dtype=torch.float64, requires_grad=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            phiT = run_differentiable(cfg, phi0, sig, steps, ckpt_every, precision=prec)
            loss = 0.5 * ((phiT - target) ** 2).sum()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        grads[prec] = sig.grad.numpy().copy()
        out[prec] = {"forward_ms": round((t1 - t0) * 1e3, 2),
                     "backward_ms": round((t2 - t1) * 1e3, 2),
                     "ms_per_adjoint_step": round((t2 - t1) * 1e3 / steps, 4),
                     "grad_finite": bool(torch.isfinite(phi0.grad).all().item()
                                         and torch.isfinite(sig.grad).all().item())}
    g64, g32 = grads["fp64"], grads["fp32"]
    out["fp32_dsigma_rel_diff_vs_fp64"] = float(np.max(np.abs(g32 - g64)) /
                                                 max(np.max(np.abs(g64)), 1e-300))
    out["adjoint_step_kernels"] = [
        time_adjoint_step("two_discs_256x256_N3_d2q9", cfg, phi),
        time_adjoint_step("many_discs_512x512_N4_d2q9", *inputs.many_discs())]
    return out


def time_adjoint_step(name, cfg, phi, reps=100):
    """The adjoint step alone (its forward-recompute and reverse kernels, one call of
    adjoint_step) timed with HIP events on the library's stream over `reps` calls, at a
    state taken after four forward steps.  Algorithmic bytes per node and step: the state
    s^t and the adjoint lambda^{t+1} read and lambda^t written, each in the FP64
    save_state64 layout (3 x its payload); the kernels also write and re-read their
    per-node intermediates, which these bytes leave out."""
    import numpy as np
    import torch
    from paper_2306_06983_amd import binding as B
    hdr = 256
    sim = B.Sim(cfg, "fp64").init(phi)
    sim.step(4)
    s0 = sim.save_state64().clone()
    payload = s0.numel() - hdr
    gen = torch.Generator(device="cpu").manual_seed(0)
    lam = torch.zeros_like(s0)
    lam[hdr:].view(torch.float64).copy_(
        torch.randn(payload // 8, generator=gen, dtype=torch.float64))
    out = torch.zeros_like(s0)
    ws = sim.adjoint_workspace()
    sim.adjoint_sigma(ws, reset=True, read=False)
    for _ in range(3):
        sim.adjoint_step(s0, lam, out, ws)
    stream = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        sim.adjoint_step(s0, lam, out, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    finite = bool(torch.isfinite(out[hdr:].view(torch.float64)).all().item())
    sim.close()
    V = int(np.prod(phi.shape[1:]))
    nbytes = 3 * payload
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": name, "ms_per_adjoint_step": round(ms, 4),
            "bytes_per_node_step": nbytes // V, "achieved_GBs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "finite": finite}


def time_oracle(cfg, phi, max_seconds=15.0, max_steps=200):
    """The oracle as it stands, on the host, single-threaded BLAS; bounded sample."""
    from threadpoolctl import threadpool_limits
    from oracle import nphase as O
    with threadpool_limits(limits=1):
        C = O.Config(cfg)
        st = O.init(C, phi)
        t0 = time.perf_counter()
        n = 0
        while n < max_steps and time.perf_counter() - t0 < max_seconds:
            st = O.step(C, st, 1)
            n += 1
        dt = time.perf_counter() - t0
    V = cfg["nx"] * cfg["ny"] * cfg["nz"]
    return dict(mlups=V * n / dt / 1e6, steps=n, seconds=dt)


def copy_rate(nbytes, reps=50):
    """GB/s of a plain device-to-device copy that reads and writes nbytes (torch's copy
    kernel): the practical streaming rate of this device at that size."""
    import torch
    src = torch.ones(max(nbytes // 8, 1), dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def copy_calibration(nbytes=256 << 20, reps=10):
    """A plain copy kernel of known size: reads and writes nbytes per launch."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 3D, 2048^2 and adjoint workloads reported beside the line")
    ap.add_argument("--only", choices=["spheres_fp64", "spheres_fp32", "bands_fp32", "bands_fp64",
                                       "rti_fp64", "rti_fp32", "adjoint_step"],
                    help="time only this other workload (adjoint_step: the adjoint step "
                         "alone on the 512^2 workload, --steps calls) and print its record")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB ten times (reference "
                         "for the memory traffic counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (--gpus {args.gpus} requested); "
              "the step is a single-GPU kernel and no multi-GPU path exists", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2306_06983_amd import inputs

    def spheres(prec, steps, warm, chain=False):
        c3, p3 = inputs.spheres(n=256)   # 256^3 D3Q19, N = 4, three drops
        label = "spheres_256x256x256_N4_d3q19"
        if chain:   # Model B with the chain-rule pair normals
            c3, label = dict(c3, pair_normals="chain"), label + "_chain_normals"
        return time_extra(c3, p3, prec, steps, warm, 3, 19, c3["n_phases"] - 1, label)

    def bands(prec, steps, warm):
        c4, p4 = inputs.layered_bands()   # 2048^2 D2Q9, N = 5 bands, gravity
        return time_extra(c4, p4, prec, steps, warm, 2, 9, c4["n_phases"] - 1,
                          "layered_bands_2048x2048_N5_d2q9")

    def rti(prec, steps, warm):
        c5, p5, _ = inputs.ternary_rti()   # 256 x 1024 D2Q9, N = 3, walls, gravity
        return time_extra(c5, p5, prec, steps, warm, 2, 9, c5["n_phases"] - 1,
                          "ternary_rti_walls_256x1024_N3_d2q9")

    if args.only == "adjoint_step":
        print(json.dumps(time_adjoint_step("many_discs_512x512_N4_d2q9", *inputs.many_discs(),
                                           reps=args.steps)))
        return 0
    if args.only:
        kind, prec = args.only.split("_")
        rec = {"spheres": spheres, "bands": bands, "rti": rti}[kind](prec, args.steps,
                                                                      args.warmup)
        print(json.dumps(rec))
        return 0

    cfg, phi = inputs.many_discs()   # 512^2, N = 4, Model B
    V = cfg["nx"] * cfg["ny"]
    d, Q, N = 2, 9, cfg["n_phases"]
    NS = N - 1
    K, W = args.steps, args.warmup

    r64 = time_gpu(cfg, phi, "fp64", K, W)
    r32 = time_gpu(cfg, phi, "fp32", K, W)
    cfgA = dict(cfg, model="A", model_a_n=1)
    rA = time_gpu(cfgA, phi, "fp64", K, W)
    rA32 = time_gpu(cfgA, phi, "fp32", K, W)
    cfgC = dict(cfg, pair_normals="chain")   # Model B, chain-rule pair normals
    rC = time_gpu(cfgC, phi, "fp64", K, W)
    rC32 = time_gpu(cfgC, phi, "fp32", K, W)

    def mlups(r):
        return V / (r["ms_per_step"] * 1e-3) / 1e6

    b64 = algorithmic_bytes_per_node(d, Q, NS, 8)
    b32 = algorithmic_bytes_per_node(d, Q, NS, 4)
    ach64 = V * b64 / (r64["ms_per_step"] * 1e-3) / 1e9
    ach32 = V * b32 / (r32["ms_per_step"] * 1e-3) / 1e9
    m64 = algorithmic_bytes_per_node_moment_form(d, Q, NS, 8)
    mgbs64 = V * m64 / (r64["ms_per_step"] * 1e-3) / 1e9
    workload = "many_discs_512x512_N4_d2q9"
    tr = measured_traffic(workload, "fp64")
    # a plain copy moving the bytes the step itself moves (the moment-form state: half
    # read, half written)
    cr64 = copy_rate(V * m64 // 2)

    # FP32 accuracy at the end of the timed run against the FP64 path (same steps)
    dphi32 = float((r32["phi"] - r64["phi"]).abs().max().item())
    drift32 = float(np.max(np.abs(r32["m1"] - r64["m0"]) / np.abs(r64["m0"])))
    drift64 = float(np.max(np.abs(r64["m1"] - r64["m0"]) / np.abs(r64["m0"])))

    line = {
        "metric": "MLUPS & % HBM peak, N-phase AC+NS LBM; FP32 vs FP64 at stated error",
        "value": round(mlups(r64), 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded discs, tanh profiles)",
        "config": {"workload": workload, "lattice": "D2Q9", "nx": 512, "ny": 512,
                   "n_phases": N, "model": "B", "solved_sets": NS, "discs": 40,
                   "steps_timed": K},
        "roofline": {"bound": "hbm", "achieved": round(ach64, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach64 / HBM_PEAK_GBS, 4),
                     "traffic": tr, "bytes_per_node_update": b64,
                     "state": "phase field stored in moment form (phi, A, D per set)",
                     "moment_form_bytes_per_node_update": m64,
                     "moment_form_GBs": round(mgbs64, 1),
                     "copy_GBs_same_bytes": round(cr64, 1),
                     "moment_form_frac_of_copy": round(mgbs64 / cr64, 4),
                     "note": "achieved/frac use the population-form bytes of the method; the "
                             "state the kernel moves is the moment form (113 MB with both "
                             "buffers), smaller than the 256 MB Infinity Cache"},
        "fp32": {"value": round(mlups(r32), 1), "ms_per_step": r32["ms_per_step"],
                 "speedup_vs_fp64": round(mlups(r32) / mlups(r64), 3),
                 "achieved_GBs": round(ach32, 1), "frac": round(ach32 / HBM_PEAK_GBS, 4),
                 "bytes_per_node_update": b32,
                 "max_abs_dphi_vs_fp64": dphi32, "mass_drift_rel": drift32},
        "model_a_n1": {"fp64_mlups": round(mlups(rA), 1), "fp32_mlups": round(mlups(rA32), 1)},
        "model_b_chain_normals": {"fp64_mlups": round(mlups(rC), 1),
                                  "fp32_mlups": round(mlups(rC32), 1)},
        "fp64_mass_drift_rel": drift64,
        "finite": bool(r64["finite"] and r32["finite"]),
    }
    if not args.no_extra:
        line["other_workloads"] = [spheres("fp64", 100, 10), spheres("fp32", 100, 10),
                                   spheres("fp64", 100, 10, chain=True),
                                   bands("fp32", 500, 50), bands("fp64", 200, 20),
                                   rti("fp64", 2000, 200),
                                   rti("fp32", 2000, 200)]
        line["rti_ternary_diagnostics"] = {"fp64": rti_diagnostics("fp64"),
                                           "fp32": rti_diagnostics("fp32")}
        line["adjoint"] = time_adjoint()
    if not args.no_cpu:
        cb = time_oracle(cfg, phi)
        line["cpu_baseline"] = {"value": round(cb["mlups"], 4), "unit": "MLUPS", "cores": 1,
                                "kind": "oracle",
                                "sample": f"{cb['steps']} steps of the same 512^2 N=4 "
                                          f"Model B workload ({cb['seconds']:.1f} s, NumPy "
                                          f"FP64, BLAS limited to 1 thread)"}
    print(json.dumps(line))
    torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
