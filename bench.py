"""Benchmark of the N-phase LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
    python bench.py --only NAME [--steps K] [--warmup W]      (one workload's record, for
                    profiling: spheres_fp64|spheres_fp32|discs_fp64|discs_fp32|bands_fp32|
                    bands_fp64|rti_fp64|rti_fp32|adjoint_step)

Headline workload: 256^3 periodic D3Q19, N = 4 phases, three seeded drops R U[20, 40] in
an ambient phase, sigma = 0.01, tau_g = 0.7, mobility 0.02, eps = 4, Model B, FP64 (the
largest single-GPU workload of the set; its state does not fit the 256 MB Infinity Cache,
so the rate is an HBM rate).  One step = one time step of every phase-field set and the
flow set over the whole grid (two launches: the moments pass and the z-marching
collide-and-stream pass), inputs resident in HBM.  Prints ONE JSON line.

value = FP64 MLUPS (node updates per second / 1e6) on that workload; the FP32
deviation-storage form is reported beside it with its error against FP64 at the workload's
5000-step horizon (measured on the 64^3 copy of the same placement), and so are the FP32
errors of the 512^2 (20000 steps) and 2048^2 (10000 steps) workloads at theirs.  Unless
--no-extra: the other workloads (512^2 N = 4 discs, LLC-resident; 64^2 touching discs;
2048^2 N = 5 layered bands; the walled ternary Rayleigh-Taylor box of Sec. 4.4; the 256^2
adjoint workload's forward), the interface locations of the Rayleigh-Taylor run, and the
differentiable 256^2 run (wall times, adjoint step kernels, adjoint vs central finite
differences).  Unless --no-cpu: the oracle timed on the host per workload (cpu_baseline).

roofline: the step is HBM-bound (no dense contraction); achieved = the method's
algorithmic bytes of one step (the population form: every persisted value read once and
written once) / the mean step time measured with HIP events on the stream the library
launches on.
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
FP32_PHI_BAR = 2e-5     # max |dphi| of the FP32 form against FP64
MASS_BAR = 1e-6         # relative per-phase mass drift
HEADLINE = "spheres_256x256x256_N4_d3q19"


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


def moments_buffer_bytes_per_node(NS, tsize):
    """D3Q19 only: the per-node moments (phi, j; FP32 residual) written by the moments pass
    and read by the collide-and-stream pass: bytes of this implementation beyond the
    algorithmic figure."""
    return 2 * NS * (4 + (1 if tsize == 4 else 0)) * tsize


# sources of the timed step kernels and of the host code that launches them (it chooses
# tiles, z-runs and the streaming form); the adjoint kernels do not enter a step
STEP_SOURCES = ("nphase_lbm.hip", "lattice.hpp", "step_kernel.hpp", "step3d_kernel.hpp", "aux_kernels.hpp",
                "dispatch.hpp", "kernels_tu.inc", "kernels_f64_d2q9.hip",
                "kernels_f32_d2q9.hip", "kernels_f64_d3q19_n2to4.hip",
                "kernels_f64_d3q19_n5.hip", "kernels_f64_d3q19_n6.hip",
                "kernels_f64_d3q19_n7.hip", "kernels_f64_d3q19_n8.hip",
                "kernels_f32_d3q19_n2to5.hip", "kernels_f32_d3q19_n6.hip",
                "kernels_f32_d3q19_n7to8.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_06983_amd", "csrc")
    for fn in STEP_SOURCES:
        h.update(open(os.path.join(csrc, fn), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per step (all launches of one step) from the committed rocprofv3
    counter summary, if it was taken with the current kernel sources (else None)."""
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


def nodes(cfg):
    return cfg["nx"] * cfg["ny"] * cfg.get("nz", 1)


def lattice_dims(cfg):
    return (2, 9) if cfg["lattice"] == "D2Q9" else (3, 19)


def solved_sets(cfg):
    return cfg["n_phases"] if cfg.get("solve_all") else cfg["n_phases"] - 1


def time_gpu(cfg, phi, precision, steps, warmup):
    """Mean step time over `steps` steps after `warmup` untimed ones, HIP events on the
    library's stream; the state after the run is checked and its phase fields kept."""
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


def record(label, cfg, precision, r, steps, note=None):
    """MLUPS and achieved GB/s of a timed run on the population-form algorithmic bytes,
    with the moment-form (and D3Q19 moments-buffer) bytes beside them."""
    d, Q = lattice_dims(cfg)
    NS = solved_sets(cfg)
    ts = 8 if precision == "fp64" else 4
    b = algorithmic_bytes_per_node(d, Q, NS, ts)
    mf = algorithmic_bytes_per_node_moment_form(d, Q, NS, ts)
    mlups = nodes(cfg) / (r["ms_per_step"] * 1e-3) / 1e6
    gbs = mlups * 1e6 * b / 1e9
    rec = {"workload": label, "precision": precision, "model": cfg["model"],
           "mlups": round(mlups, 1), "ms_per_step": round(r["ms_per_step"], 5),
           "steps_timed": steps, "bytes_per_node_update": b, "achieved_GBs": round(gbs, 1),
           "frac": round(gbs / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic(label, precision), "finite": bool(r["finite"]),
           "moment_form_bytes_per_node_update": mf,
           "moment_form_GBs": round(mlups * 1e6 * mf / 1e9, 1),
           # per phase after warm-up + timed steps: Y_av, Y_min, Y_max (rows / z planes)
           "interface_locations": {"Y_av": [round(float(v), 3) for v in r["locations"][0]],
                                   "Y_min": [int(v) for v in r["locations"][1]],
                                   "Y_max": [int(v) for v in r["locations"][2]]}}
    if d == 3:
        rec["moments_buffer_bytes_per_node_update"] = moments_buffer_bytes_per_node(NS, ts)
    if note:
        rec["note"] = note
    return rec


def perturbed(phi, seed=1, rel=2.2e-16):
    """phi0 with the evolved phases multiplied by (1 + rel N(0, 1)) (one rounding) and the
    last phase rebuilt as 1 - sum."""
    import numpy as np
    rng = np.random.default_rng(seed)
    p = phi.copy()
    for k in range(p.shape[0] - 1):
        p[k] = p[k] * (1 + rel * rng.standard_normal(p[k].shape))
    p[-1] = 1 - p[:-1].sum(0)
    return p


def fp32_accuracy(label, cfg, phi, steps):
    """The FP32 form against the FP64 path at a workload's own horizon: max |dphi| and its
    99.9 % quantile over all nodes and phases, the FP64 path's own spread under a
    one-rounding perturbation of phi0 (the envelope no implementation summing in another
    order can beat), per-phase relative mass drift of both, and whether the bars
    (max |dphi| <= 2e-5, mass drift <= 1e-6) are met.  The FP64 GPU path is the reference
    here: beyond oracle-feasible lengths it stands for the oracle, against which it is
    checked on prefixes by the parity tests."""
    import numpy as np
    import torch
    from paper_2306_06983_amd import binding as B

    def run(prec, phi0):
        s = B.Sim(cfg, prec).init(phi0)
        m0 = s.mass()
        s.step(steps)
        ph = s.fields()[0]
        m1 = s.mass()
        ok = s.check()
        s.close()
        return ph, m0, m1, ok

    t0 = time.perf_counter()
    ph64, m0, m1_64, ok64 = run("fp64", phi)
    ph64b = run("fp64", perturbed(phi))[0]
    ph32, m0_32, m1_32, ok32 = run("fp32", phi)
    d = (ph32 - ph64).abs().flatten()
    k = max(1, int(np.ceil(1e-3 * d.numel())))
    p999 = float(torch.topk(d, k).values.min().item())
    dmax = float(d.max().item())
    env = float((ph64b - ph64).abs().max().item())
    drift32 = float(np.max(np.abs(m1_32 - m0) / np.abs(m0)))
    drift64 = float(np.max(np.abs(m1_64 - m0) / np.abs(m0)))
    del ph64, ph64b, ph32, d
    torch.cuda.empty_cache()
    return {"workload": label, "steps": steps, "reference": "FP64 GPU path",
            "max_abs_dphi": dmax, "p999_abs_dphi": p999,
            "fp64_one_rounding_envelope": env,
            "max_over_envelope": round(dmax / env, 3) if env > 0 else None,
            "mass_drift_rel_fp32": drift32, "mass_drift_rel_fp64": drift64,
            "bar_max_abs_dphi": FP32_PHI_BAR, "bar_mass_drift_rel": MASS_BAR,
            "max_exceeds_bar": dmax > FP32_PHI_BAR, "p999_exceeds_bar": p999 > FP32_PHI_BAR,
            "mass_exceeds_bar": drift32 > MASS_BAR,
            "finite": bool(ok64 and ok32), "wall_s": round(time.perf_counter() - t0, 1)}


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


def _gpu_loss(cfg, phi, target, steps):
    from paper_2306_06983_amd import binding as B
    s = B.Sim(cfg, "fp64").init(phi)
    s.step(steps)
    ph = s.fields()[0]
    out = 0.5 * float(((ph - target) ** 2).sum().item())
    s.close()
    return out


def adjoint_vs_fd(cfg, phi, pairs, target, grads, steps, rels=(1e-4, 1e-5)):
    """dL/dsigma_pq of the adjoint against central differences of the FP64 forward (the
    path the parity tests tie to the oracle) at two step sizes h = rel * sigma_pq; the
    difference quotients have converged where the two agree."""
    from paper_2306_06983_amd import inputs
    out = []
    for k in range(len(pairs)):
        fds = []
        for rel in rels:
            h = rel * pairs[k]
            pp, pm = pairs.copy(), pairs.copy()
            pp[k] += h
            pm[k] -= h
            fds.append((_gpu_loss(inputs.with_sigma_pairs(cfg, pp), phi, target, steps) -
                        _gpu_loss(inputs.with_sigma_pairs(cfg, pm), phi, target, steps)) / (2 * h))
        out.append({"pair": k, "adjoint": float(grads[k]), "fd_h": fds[0], "fd_h_over_10": fds[1],
                    "rel_err_vs_fd_h": abs(grads[k] - fds[0]) / max(abs(fds[0]), 1e-300),
                    "fd_converged_rel": abs(fds[0] - fds[1]) / max(abs(fds[0]), 1e-300)})
    return out


def time_adjoint(steps=25, ckpt_every=10, long_steps=400, long_ckpt=50):
    """Differentiable run on the 256^2 N = 3 touching discs, loss = L2 misfit of phi(T) to
    a run with sigma_pq scaled by seeded U[0.8, 1.2]: wall time of the forward (with
    checkpoints) and of the backward (segment recompute + hand-written adjoint steps) for
    the FP64 form and for the FP32 form (FP32 forward, FP64 adjoint steps along it), each
    after an untimed warm-up run; max |dL/dsigma(FP32) - dL/dsigma(FP64)| relative to
    max |dL/dsigma(FP64)|; dL/dsigma against central differences at T = 25 (where the
    difference quotients converge) and, as a record of the conditioning, at T = 400 with
    checkpoints every 50 steps (the workload's own horizon, where they do not)."""
    import numpy as np
    import torch
    from paper_2306_06983_amd import binding as B
    from paper_2306_06983_amd import inputs
    from paper_2306_06983_amd.autograd import run_differentiable
    cfg, phi = inputs.two_discs(scale=4)
    pairs = inputs.sigma_pairs(cfg)
    rng = np.random.default_rng(5)
    cfg_t = inputs.with_sigma_pairs(cfg, pairs * rng.uniform(0.8, 1.2, size=len(pairs)))

    def target_at(T):
        tsim = B.Sim(cfg_t, "fp64").init(phi)
        tsim.step(T)
        tg = tsim.fields()[0].clone()
        tsim.close()
        return tg

    def grad(T, ck, prec, reps=2):
        for rep in range(reps):   # the first run warms up the allocator and the kernels
            phi0 = torch.tensor(phi, dtype=torch.float64, device="cuda:0", requires_grad=True)
            sig = torch.tensor(pairs, dtype=torch.float64, requires_grad=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            phiT = run_differentiable(cfg, phi0, sig, T, ck, precision=prec)
            loss = 0.5 * ((phiT - tgt[T]) ** 2).sum()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        ok = bool(torch.isfinite(phi0.grad).all().item() and torch.isfinite(sig.grad).all().item())
        return sig.grad.numpy().copy(), t1 - t0, t2 - t1, ok

    tgt = {steps: target_at(steps), long_steps: target_at(long_steps)}
    out = {"workload": "two_discs_256x256_N3_d2q9_adjoint", "steps": steps,
           "ckpt_every": ckpt_every}
    grads = {}
    for prec in ("fp64", "fp32"):
        g, tf, tb, ok = grad(steps, ckpt_every, prec)
        grads[prec] = g
        out[prec] = {"forward_ms": round(tf * 1e3, 2), "backward_ms": round(tb * 1e3, 2),
                     "ms_per_adjoint_step": round(tb * 1e3 / steps, 4), "grad_finite": ok}
    g64, g32 = grads["fp64"], grads["fp32"]
    out["fp32_dsigma_rel_diff_vs_fp64"] = float(np.max(np.abs(g32 - g64)) /
                                                 max(np.max(np.abs(g64)), 1e-300))
    fd = adjoint_vs_fd(cfg, phi, pairs, tgt[steps], g64, steps)
    out["fd_check"] = {"steps": steps, "pairs": fd,
                       "max_rel_err": max(r["rel_err_vs_fd_h"] for r in fd), "bar": 1e-4}
    gL, tf, tb, ok = grad(long_steps, long_ckpt, "fp64", reps=1)
    fdL = adjoint_vs_fd(cfg, phi, pairs, tgt[long_steps], gL, long_steps)
    out["horizon_400"] = {"steps": long_steps, "ckpt_every": long_ckpt,
                          "backward_ms": round(tb * 1e3, 2), "grad_finite": ok, "pairs": fdL,
                          "note": "difference quotients at h and h/10 disagree: the discrete "
                                  "map's derivative is not bounded at this horizon"}
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


def time_oracle(cfg, phi, max_steps, max_seconds):
    """The oracle as it stands, on the host, BLAS limited to one thread; at most
    max_steps steps, stopping after the first step that ends past max_seconds."""
    from threadpoolctl import threadpool_limits
    from oracle import nphase as O
    with threadpool_limits(limits=1):
        C = O.Config(cfg)
        st = O.init(C, phi)
        t0 = time.perf_counter()
        n = 0
        while n < max_steps and (n == 0 or time.perf_counter() - t0 < max_seconds):
            st = O.step(C, st, 1)
            n += 1
        dt = time.perf_counter() - t0
    return dict(mlups=nodes(cfg) * n / dt / 1e6, steps=n, seconds=dt)


def affinity():
    try:
        cpus = sorted(os.sched_getaffinity(0))
    except AttributeError:
        return None
    runs, start = [], None
    for i, c in enumerate(cpus):
        if start is None:
            start = c
        if i + 1 == len(cpus) or cpus[i + 1] != c + 1:
            runs.append(f"{start}-{c}" if c != start else f"{c}")
            start = None
    return {"count": len(cpus), "set": ",".join(runs)}


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


def workloads():
    """label -> (generator, note) of every timed workload."""
    from paper_2306_06983_amd import inputs
    return {
        HEADLINE: (lambda: inputs.spheres(n=256), None),
        "spheres_256x256x256_N4_d3q19_chain_normals":
            (lambda: (lambda c, p: (dict(c, pair_normals="chain"), p))(*inputs.spheres(n=256)),
             "Model B with the chain-rule pair normals"),
        "many_discs_512x512_N4_d2q9":
            (lambda: inputs.many_discs(),
             "LLC-resident: the moment-form state (113 MB FP64 with both buffers) fits the "
             "256 MB Infinity Cache, so this is not an HBM rate"),
        "many_discs_512x512_N4_d2q9_model_a_n1":
            (lambda: inputs.many_discs(model="A", model_a_n=1), "LLC-resident"),
        "layered_bands_2048x2048_N5_d2q9": (lambda: inputs.layered_bands(), None),
        "two_discs_64x64_N3_d2q9":
            (lambda: inputs.two_discs(), "correctness workload; 4096 nodes: launch-latency bound"),
        "two_discs_256x256_N3_d2q9":
            (lambda: inputs.two_discs(scale=4), "forward of the adjoint workload; cache-resident"),
        "ternary_rti_walls_256x1024_N3_d2q9":
            (lambda: inputs.ternary_rti()[:2], "walls and gravity; LLC-resident"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads, the long-horizon accuracy runs and the "
                         "adjoint reported beside the line")
    ap.add_argument("--only", choices=["spheres_fp64", "spheres_fp32", "discs_fp64",
                                       "discs_fp32", "bands_fp32", "bands_fp64", "rti_fp64",
                                       "rti_fp32", "adjoint_step"],
                    help="time only this workload (adjoint_step: the adjoint step alone on "
                         "the 512^2 workload, --steps calls) and print its record")
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

    W = workloads()
    K, Wm = args.steps, args.warmup
    if args.only == "adjoint_step":
        print(json.dumps(time_adjoint_step("many_discs_512x512_N4_d2q9", *inputs.many_discs(),
                                           reps=args.steps)))
        return 0
    if args.only:
        kind, prec = args.only.split("_")
        label = {"spheres": HEADLINE, "discs": "many_discs_512x512_N4_d2q9",
                 "bands": "layered_bands_2048x2048_N5_d2q9",
                 "rti": "ternary_rti_walls_256x1024_N3_d2q9"}[kind]
        cfg, phi = W[label][0]()
        print(json.dumps(record(label, cfg, prec, time_gpu(cfg, phi, prec, K, Wm), K)))
        return 0

    # ---- headline: 256^3 D3Q19 N = 4 three drops, FP64, FP32 beside it
    cfg, phi = W[HEADLINE][0]()
    V = nodes(cfg)
    d, Q = 3, 19
    NS = solved_sets(cfg)
    r64 = time_gpu(cfg, phi, "fp64", K, Wm)
    r32 = time_gpu(cfg, phi, "fp32", K, Wm)
    rec64 = record(HEADLINE, cfg, "fp64", r64, K)
    rec32 = record(HEADLINE, cfg, "fp32", r32, K)
    del phi
    b64 = algorithmic_bytes_per_node(d, Q, NS, 8)
    moved64 = (algorithmic_bytes_per_node_moment_form(d, Q, NS, 8) +
               moments_buffer_bytes_per_node(NS, 8))
    cr = copy_rate(V * moved64 // 2)   # a plain copy of the bytes one step moves
    mlups64 = rec64["mlups"]
    line = {
        "metric": "MLUPS & % HBM peak, N-phase AC+NS LBM; FP32 vs FP64 at stated error",
        "value": mlups64,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded spheres, tanh profiles)",
        "config": {"workload": HEADLINE, "lattice": "D3Q19", "nx": 256, "ny": 256, "nz": 256,
                   "n_phases": 4, "model": "B", "solved_sets": NS, "drops": 3,
                   "steps_timed": K},
        "roofline": {"bound": "hbm", "achieved": rec64["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": rec64["frac"], "traffic": rec64["traffic"],
                     "kernel": "one step = nphase_moments3d_kernel + nphase_step3d_kernel",
                     "bytes_per_node_update": b64, "nodes_per_launch": V,
                     "moment_form_bytes_per_node_update": rec64["moment_form_bytes_per_node_update"],
                     "moments_buffer_bytes_per_node_update": rec64["moments_buffer_bytes_per_node_update"],
                     "moved_GBs": round(V * moved64 / (r64["ms_per_step"] * 1e-3) / 1e9, 1),
                     "copy_GBs_same_bytes": round(cr, 1),
                     "note": "achieved/frac on the population-form bytes of the method (the "
                             "algorithmic figure); the kernels keep the phase field in moment "
                             "form and add the moments buffer, whose bytes moved_GBs counts; "
                             "traffic = rocprofv3 FETCH_SIZE + WRITE_SIZE of one step (both "
                             "launches), scaled by the plain-copy calibration, or null when "
                             "taken with other kernel sources"},
        "fp32": {"value": rec32["mlups"], "ms_per_step": r32["ms_per_step"],
                 "speedup_vs_fp64": round(rec32["mlups"] / mlups64, 3),
                 "achieved_GBs": rec32["achieved_GBs"], "frac": rec32["frac"],
                 "bytes_per_node_update": rec32["bytes_per_node_update"],
                 "traffic": rec32["traffic"]},
        "fp64_mass_drift_rel": float(np.max(np.abs(r64["m1"] - r64["m0"]) / np.abs(r64["m0"]))),
        "finite": bool(r64["finite"] and r32["finite"]),
    }
    del r64, r32
    torch.cuda.empty_cache()

    if not args.no_extra:
        # FP32 against FP64 at each workload's own horizon; the 256^3 workload's at 5000
        # steps on its 64^3 copy (the same placement scaled by 1/4)
        c3s, p3s = inputs.spheres(n=64, scale=0.25)
        acc3 = fp32_accuracy("spheres_64x64x64_N4_d3q19 (copy of the headline)", c3s, p3s, 5000)
        acc3["fp32_speedup_on_headline"] = line["fp32"]["speedup_vs_fp64"]
        line["fp32"]["accuracy"] = acc3
        c2, p2 = inputs.many_discs()
        c4, p4 = inputs.layered_bands()
        line["fp32_accuracy_other"] = [fp32_accuracy("many_discs_512x512_N4_d2q9", c2, p2, 20000),
                                       fp32_accuracy("layered_bands_2048x2048_N5_d2q9", c4, p4, 10000)]
        del p2, p4
        plan = [("spheres_256x256x256_N4_d3q19_chain_normals", "fp64", 20, 5),
                ("many_discs_512x512_N4_d2q9", "fp64", 2000, 200),
                ("many_discs_512x512_N4_d2q9", "fp32", 2000, 200),
                ("many_discs_512x512_N4_d2q9_model_a_n1", "fp64", 2000, 200),
                ("layered_bands_2048x2048_N5_d2q9", "fp32", 500, 50),
                ("layered_bands_2048x2048_N5_d2q9", "fp64", 200, 20),
                ("two_discs_64x64_N3_d2q9", "fp64", 2000, 200),
                ("two_discs_256x256_N3_d2q9", "fp64", 2000, 200),
                ("two_discs_256x256_N3_d2q9", "fp32", 2000, 200),
                ("ternary_rti_walls_256x1024_N3_d2q9", "fp64", 2000, 200),
                ("ternary_rti_walls_256x1024_N3_d2q9", "fp32", 2000, 200)]
        others = []
        for label, prec, k, w in plan:
            gen, note = W[label]
            c, p = gen()
            others.append(record(label, c, prec, time_gpu(c, p, prec, k, w), k, note))
        line["other_workloads"] = others
        for o in others:   # the FP32/FP64 speedup beside each accuracy record
            for a in line["fp32_accuracy_other"]:
                if a["workload"] == o["workload"] and o["precision"] == "fp32":
                    f64 = [x for x in others if x["workload"] == o["workload"] and
                           x["precision"] == "fp64"]
                    if f64:
                        a["fp32_speedup"] = round(o["mlups"] / f64[0]["mlups"], 3)
        line["rti_ternary_diagnostics"] = {"fp64": rti_diagnostics("fp64"),
                                           "fp32": rti_diagnostics("fp32")}
        line["adjoint"] = time_adjoint()

    if not args.no_cpu:
        # the oracle on the host, one core, bounded samples of each workload; the 256^3
        # state does not fit a NumPy oracle run, so the headline's sample is its 64^3 copy
        gpu_rate = {(o["workload"], o["precision"]): o["mlups"]
                    for o in line.get("other_workloads", [])}
        gpu_rate[(HEADLINE, "fp64")] = mlups64
        samples = [("two_discs_64x64_N3_d2q9", inputs.two_discs(), 2000, 10.0),
                   ("spheres_64x64x64_N4_d3q19", inputs.spheres(n=64, scale=0.25), 10, 10.0),
                   ("many_discs_512x512_N4_d2q9", inputs.many_discs(), 20, 10.0),
                   ("layered_bands_2048x2048_N5_d2q9", inputs.layered_bands(), 3, 10.0),
                   ("two_discs_256x256_N3_d2q9", inputs.two_discs(scale=4), 50, 10.0)]
        per = []
        for label, (c, p), nmax, tmax in samples:
            cb = time_oracle(c, p, nmax, tmax)
            g = mlups64 if label.startswith("spheres") else gpu_rate.get((label, "fp64"))
            per.append({"workload": label, "oracle_mlups": round(cb["mlups"], 4),
                        "steps": cb["steps"], "seconds": round(cb["seconds"], 1),
                        "gpu_fp64_mlups": g,
                        "gpu_over_oracle": round(g / cb["mlups"], 1) if g else None})
        head = per[1]
        line["cpu_baseline"] = {
            "value": head["oracle_mlups"], "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{head['steps']} steps of the 64^3 copy of the 256^3 three-drop "
                      f"workload ({head['seconds']} s; NumPy FP64, BLAS limited to 1 thread; "
                      f"the 256^3 state itself does not fit a NumPy oracle run)",
            "os_cpu_count": os.cpu_count(), "affinity": affinity(),
            "per_workload": per}
    print(json.dumps(line))
    torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
