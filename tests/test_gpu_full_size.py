"""Parity at the full sizes of the 3D and 2048^2 workloads, in the launch configuration the
benchmark times, on sampled outputs the oracle computes one by one.

One step of the method at a node depends on the state within four nodes of it (pull from
the upwind neighbour, whose collision uses gradients of phi and of the pair fractions at
radius two and the correction force from m_phi at radius one, rebuilt from the state one
node further out).  So the GPU state after step t is exported (FP64 populations,
save_state64), a periodic patch of P nodes per axis is cut around each sampled node, the
oracle advances the patch by one step, and the nodes at least four away from the patch
border are compared with the GPU's own export after step t + 1 (g_0 excluded: it is not
stored).  Sampled nodes: interface nodes (0.2 < phi_0 < 0.8) and seeded random ones.

Bars: FP64 every array within 1e-12 of its largest entry.  FP32 (the 2048^2 bands run in
FP32): the step of the FP32 state against the FP64 oracle step of the same state, i.e. one
step of FP32 rounding: populations and phi^{t-1} within 1e-6 absolute (about 16 units of
FP32 rounding at magnitude 1/2), u and m_phi within 1e-4 of their largest entry (m_phi: of
the magnitude M max(rho_p) / eps of the terms it sums)."""
import numpy as np
import pytest

from oracle import nphase as O
from paper_2306_06983_amd import inputs

pytestmark = pytest.mark.gpu

HDR = 256
R_DEP = 4


def _views(buf, cfg):
    """Device views [component, *grid] of a save_state64 payload."""
    import torch
    d = 2 if cfg["lattice"] == "D2Q9" else 3
    Q = 9 if d == 2 else 19
    N = cfg["n_phases"]
    NS = N if cfg.get("solve_all", False) else N - 1
    grid = (cfg["ny"], cfg["nx"]) if d == 2 else (cfg["nz"], cfg["ny"], cfg["nx"])
    V = int(np.prod(grid))
    pay = buf[HDR:].view(torch.float64)
    out, o = {}, 0
    for key, n in (("f", NS * Q), ("g", Q - 1), ("u_prev", d), ("phi_prev", NS),
                   ("mphi_prev", d)):
        out[key] = pay[o:o + n * V].view((n,) + grid)
        o += n * V
    out["f"] = out["f"].view((NS, Q) + grid)
    return out, d, Q


def _cut(t, centre, P, grid):
    """Periodic patch of P nodes per axis centred on `centre` (grid order), to host."""
    import torch
    idx = [torch.tensor([(c - P // 2 + k) % n for k in range(P)], device=t.device)
           for c, n in zip(centre, grid)]
    lead = t.dim() - len(grid)
    for a, ix in enumerate(idx):
        t = torch.index_select(t, lead + a, ix)
    return t.cpu().numpy()


def _rho_bar(cfg, phi0):
    """Domain-mean density of the initial state (the gravity reference)."""
    phi0 = np.asarray(phi0, dtype=np.float64)
    if not cfg.get("solve_all", False):
        phi0 = np.concatenate([phi0[:-1], (1.0 - phi0[:-1].sum(0))[None]], axis=0)
    rho = sum(cfg["rho"][p] * phi0[p] for p in range(phi0.shape[0]))
    return float(rho.mean())


def _sampled_parity(cfg, phi0, precision, P, n_samples, warm_steps=2, seed=0):
    import torch
    from paper_2306_06983_amd import binding as B
    s = B.Sim(cfg, precision).init(phi0)
    s.step(warm_steps)
    ph = s.fields()[0]
    buf_t = s.save_state64().clone()
    s.step(1)
    buf_t1 = s.save_state64()
    torch.cuda.synchronize()
    grid = tuple(ph.shape[1:])
    # interface nodes spread over the grid, plus seeded random nodes
    iface = torch.nonzero((ph[0] > 0.2) & (ph[0] < 0.8))
    rng = np.random.default_rng(seed)
    picks = [tuple(int(v) for v in iface[int(k)].tolist())
             for k in rng.choice(iface.shape[0], size=n_samples, replace=False)]
    picks += [tuple(int(rng.integers(0, n)) for n in grid) for _ in range(2)]
    vt, d, Q = _views(buf_t, cfg)
    vt1, _, _ = _views(buf_t1, cfg)
    pcfg = dict(cfg, nx=P, ny=P, nz=P if d == 3 else 1)
    C = O.Config(pcfg)
    inner = (slice(None),) + tuple(slice(R_DEP, P - R_DEP) for _ in range(d))
    err, scale = {}, {}
    for centre in picks:
        st = {k: _cut(v, centre, P, grid) for k, v in vt.items()}
        st["g"] = np.concatenate([np.zeros((1,) + st["g"].shape[1:]), st["g"]], axis=0)
        st["rho_bar"] = _rho_bar(cfg, phi0)
        st["t"] = warm_steps
        o = O.step(C, st, 1)
        for k, v in vt1.items():
            got = _cut(v, centre, P, grid)
            want = o[k][1:] if k == "g" else o[k]
            if k == "f":
                got, want = got.reshape((-1,) + got.shape[2:]), want.reshape((-1,) + want.shape[2:])
            err[k] = max(err.get(k, 0.0), float(np.abs(got[inner] - want[inner]).max()))
            scale[k] = max(scale.get(k, 0.0), float(np.abs(want[inner]).max()))
    s.close()
    # relative to the largest entry over all patches (a bulk patch can be all but zero in
    # u and m_phi); m_phi = -M sum_p rho_p (grad phi_p - R_p) is a sum whose terms reach
    # M max(rho_p) / eps (the largest tanh-profile gradient is 1/eps), which is zero with
    # equal densities: it is measured against that magnitude too.  FP32 populations and phi
    # absolute.
    scale["mphi_prev"] = max(scale["mphi_prev"], cfg["mobility"] * max(cfg["rho"]) / cfg["eps"])
    worst = {k: err[k] if (precision == "fp32" and k in ("f", "g", "phi_prev"))
             else err[k] / max(scale[k], 1e-300) for k in err}
    return worst, len(picks)


def _check(worst, precision):
    if precision == "fp64":
        for k, e in worst.items():
            assert e <= 1e-12, (k, e)
    else:
        for k in ("f", "g", "phi_prev"):
            assert worst[k] <= 1e-6, (k, worst[k])
        for k in ("u_prev", "mphi_prev"):
            assert worst[k] <= 1e-4, (k, worst[k])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_spheres_256_cubed_sampled(precision):
    """256^3 D3Q19 N = 4 three drops (Model B), the benchmark's 3D workload."""
    cfg, phi = inputs.spheres(n=256)
    worst, n = _sampled_parity(cfg, phi, precision, P=14, n_samples=6)
    print(f"  256^3 {precision}: {n} patches, worst {worst}")
    _check(worst, precision)


def test_bands_2048_squared_sampled():
    """2048^2 D2Q9 N = 5 layered bands with gravity, FP32 (the precision it is timed in)."""
    cfg, phi = inputs.layered_bands()
    worst, n = _sampled_parity(cfg, phi, "fp32", P=16, n_samples=8)
    print(f"  2048^2 fp32: {n} patches, worst {worst}")
    _check(worst, "fp32")
