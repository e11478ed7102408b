"""Thin Python binding of libnphase_lbm.so (the C ABI in include/nphase_lbm.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch provides the device memory (the caller-owned workspace, input and output
tensors) and the stream (torch's current stream on the device).  There is no fallback:
if the library is missing or cannot be loaded, every entry point raises.
"""
import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnphase_lbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "nphase_lbm.h")

NPHASE_OK, NPHASE_EINVAL, NPHASE_ENOMEM, NPHASE_EDEVICE = 0, -1, -2, -3
NPHASE_ENAN, NPHASE_ESTATE, NPHASE_ENOTSUP = -4, -5, -6
D2Q9, D3Q19 = 0, 1
MODEL_A, MODEL_B = 0, 1
FP64, FP32 = 0, 1
MAX_N = 8


class Params(ctypes.Structure):
    """Mirror of nphase_lbm_params."""
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("lattice", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("n_phases", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("model_a_n", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("solve_all", ctypes.c_int32),
        ("sigma", ctypes.c_double * (MAX_N * MAX_N)),
        ("rho", ctypes.c_double * MAX_N),
        ("tau_g", ctypes.c_double * MAX_N),
        ("mobility", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("gravity", ctypes.c_double * 3),
        ("walls", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("contact_cos", ctypes.c_double * MAX_N),
        ("pair_normals", ctypes.c_int32),
        ("pad1", ctypes.c_int32),
    ]


class NPhaseError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load():
    """Load the shared library (raises if it is missing: no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2306_06983_amd.build` (HIP, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Params)
    vp, sz, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64
    sig = {
        "nphase_lbm_workspace_bytes": [P, ctypes.POINTER(sz)],
        "nphase_lbm_create": [P, vp, sz, vp, ctypes.POINTER(vp)],
        "nphase_lbm_init": [vp, vp],
        "nphase_lbm_step": [vp, i64],
        "nphase_lbm_fields": [vp, vp, vp, vp],
        "nphase_lbm_mass": [vp, ctypes.POINTER(ctypes.c_double)],
        "nphase_lbm_check": [vp, ctypes.POINTER(ctypes.c_int)],
        "nphase_lbm_interface_locations": [vp, vp, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32)],
        "nphase_lbm_interface_locations_noalloc": [
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
            vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
            ctypes.POINTER(ctypes.c_int32)],
        "nphase_lbm_time": [vp, ctypes.POINTER(i64)],
        "nphase_lbm_state_bytes": [vp, ctypes.POINTER(sz)],
        "nphase_lbm_save_state": [vp, vp],
        "nphase_lbm_load_state": [vp, vp],
        "nphase_lbm_state64_bytes": [vp, ctypes.POINTER(sz)],
        "nphase_lbm_save_state64": [vp, vp],
        "nphase_lbm_destroy": [vp],
        "nphase_lbm_adjoint_workspace_bytes": [vp, ctypes.POINTER(sz)],
        "nphase_lbm_adjoint_seed": [vp, vp, vp],
        "nphase_lbm_adjoint_step": [vp, vp, vp, vp, vp, sz],
        "nphase_lbm_adjoint_sigma": [vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int],
        "nphase_lbm_adjoint_init": [vp, vp, vp, sz, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.nphase_lbm_last_error.argtypes = [vp]
    lib.nphase_lbm_last_error.restype = ctypes.c_char_p
    lib.nphase_lbm_strerror.argtypes = [ctypes.c_int]
    lib.nphase_lbm_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def header_functions():
    """Names of the functions declared in include/nphase_lbm.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(nphase_lbm_[a-z_]+)\s*\(", txt)))


def make_params(cfg, precision="fp64"):
    """nphase_lbm_params from a configuration dictionary (keys as in inputs.base_cfg)."""
    p = Params()
    p.struct_size = ctypes.sizeof(Params)
    p.lattice = {"D2Q9": D2Q9, "D3Q19": D3Q19}[cfg["lattice"]]
    p.nx, p.ny, p.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg.get("nz", 1))
    N = int(cfg["n_phases"])
    p.n_phases = N
    p.model = {"A": MODEL_A, "B": MODEL_B}[cfg["model"]]
    p.model_a_n = int(cfg.get("model_a_n", 1))
    p.precision = {"fp64": FP64, "fp32": FP32}[precision]
    p.solve_all = 1 if cfg.get("solve_all", False) else 0
    sig = np.asarray(cfg["sigma"], dtype=np.float64).reshape(N, N)
    for i in range(N):
        for j in range(N):
            p.sigma[i * MAX_N + j] = float(sig[i, j])
        p.rho[i] = float(cfg["rho"][i])
        p.tau_g[i] = float(cfg["tau_g"][i])
    p.mobility = float(cfg["mobility"])
    p.eps = float(cfg["eps"])
    g = list(cfg.get("gravity", [0.0, 0.0, 0.0])) + [0.0, 0.0, 0.0]
    for d in range(3):
        p.gravity[d] = float(g[d])
    p.walls = 1 if cfg.get("walls", False) else 0
    for i, c in enumerate(cfg.get("contact_cos", [])):
        p.contact_cos[i] = float(c)
    p.pair_normals = {"stencil": 0, "chain": 1}[cfg.get("pair_normals", "stencil")]
    return p


def interface_locations_noalloc(phi, lattice):
    """(Y_av, Y_min, Y_max) of an FP64 CUDA tensor phi [N, *grid] through the handle-free
    entry point that allocates nothing (its reduction scratch is a static device array of
    the library), on torch's current stream of phi's device."""
    import torch
    lib = load()
    if not (phi.is_cuda and phi.dtype == torch.float64):
        raise ValueError("phi must be an FP64 CUDA tensor")
    phi = phi.contiguous()
    N = int(phi.shape[0])
    if lattice == "D2Q9":
        ny, nx = phi.shape[1:]
        nz = 1
    else:
        nz, ny, nx = phi.shape[1:]
    av = (ctypes.c_double * max(N, 1))()
    lo = (ctypes.c_int32 * max(N, 1))()
    hi = (ctypes.c_int32 * max(N, 1))()
    with torch.cuda.device(phi.device):
        stream = torch.cuda.current_stream(phi.device)
        rc = lib.nphase_lbm_interface_locations_noalloc(
            {"D2Q9": D2Q9, "D3Q19": D3Q19}[lattice], int(nx), int(ny), int(nz), N,
            ctypes.c_void_p(phi.data_ptr()), ctypes.c_void_p(stream.cuda_stream), av, lo, hi)
    if rc != NPHASE_OK:
        raise NPhaseError(rc, lib.nphase_lbm_strerror(rc).decode())
    return (np.array(av[:N], dtype=np.float64), np.array(lo[:N], dtype=np.int64),
            np.array(hi[:N], dtype=np.int64))


class Sim:
    """One simulation handle on a CUDA/HIP device, bound to torch's current stream."""

    def __init__(self, cfg, precision="fp64", device="cuda:0"):
        import torch
        self.torch = torch
        self.lib = load()
        self.cfg = cfg
        self.precision = precision
        self.params = make_params(cfg, precision)
        self.device = torch.device(device)
        self.N = int(cfg["n_phases"])
        self.d = 2 if cfg["lattice"] == "D2Q9" else 3
        nx, ny, nz = self.params.nx, self.params.ny, self.params.nz
        self.grid = (ny, nx) if self.d == 2 else (nz, ny, nx)
        nbytes = ctypes.c_size_t()
        self._rc(self.lib.nphase_lbm_workspace_bytes(ctypes.byref(self.params),
                                                     ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        self._rc(self.lib.nphase_lbm_create(ctypes.byref(self.params),
                                            ctypes.c_void_p(self._ws_ptr),
                                            self.ws_bytes,
                                            ctypes.c_void_p(self.stream.cuda_stream),
                                            ctypes.byref(h)))
        self.h = h

    def _rc(self, rc, h=None):
        if rc != NPHASE_OK:
            msg = self.lib.nphase_lbm_strerror(rc).decode()
            hh = h if h is not None else getattr(self, "h", None)
            if hh:
                msg += ": " + self.lib.nphase_lbm_last_error(hh).decode()
            raise NPhaseError(rc, msg)

    def init(self, phi0):
        t = self.torch
        x = t.as_tensor(np.asarray(phi0) if not t.is_tensor(phi0) else phi0)
        x = x.to(device=self.device, dtype=t.float64).contiguous()
        if tuple(x.shape) != (self.N,) + self.grid:
            raise ValueError(f"phi0 shape {tuple(x.shape)} != {(self.N,) + self.grid}")
        self._rc(self.lib.nphase_lbm_init(self.h, ctypes.c_void_p(x.data_ptr())))
        return self

    def step(self, n=1):
        self._rc(self.lib.nphase_lbm_step(self.h, int(n)))
        return self

    def fields(self):
        """(phi [N, *grid], u [d, *grid], P [*grid]) as FP64 device tensors."""
        t = self.torch
        phi = t.empty((self.N,) + self.grid, dtype=t.float64, device=self.device)
        u = t.empty((self.d,) + self.grid, dtype=t.float64, device=self.device)
        P = t.empty(self.grid, dtype=t.float64, device=self.device)
        self._rc(self.lib.nphase_lbm_fields(self.h, ctypes.c_void_p(phi.data_ptr()),
                                            ctypes.c_void_p(u.data_ptr()),
                                            ctypes.c_void_p(P.data_ptr())))
        return phi, u, P

    def mass(self):
        out = (ctypes.c_double * self.N)()
        self._rc(self.lib.nphase_lbm_mass(self.h, out))
        return np.array(out[:], dtype=np.float64)

    def interface_locations(self, phi=None):
        """(Y_av [N] float, Y_min [N] int, Y_max [N] int) of FP64 device phase fields
        phi [N, *grid] (default: the current fields); heights are row (2D) / plane (3D)
        indices."""
        if phi is None:
            phi = self.fields()[0]
        phi = phi.contiguous()
        assert phi.dtype == self.torch.float64 and phi.is_cuda
        assert tuple(phi.shape) == (self.N,) + self.grid
        av = (ctypes.c_double * self.N)()
        lo = (ctypes.c_int32 * self.N)()
        hi = (ctypes.c_int32 * self.N)()
        self._rc(self.lib.nphase_lbm_interface_locations(self.h, ctypes.c_void_p(phi.data_ptr()),
                                                         av, lo, hi))
        return (np.array(av[:], dtype=np.float64), np.array(lo[:], dtype=np.int64),
                np.array(hi[:], dtype=np.int64))

    def check(self):
        ok = ctypes.c_int(0)
        rc = self.lib.nphase_lbm_check(self.h, ctypes.byref(ok))
        if rc == NPHASE_ENAN:
            return False
        self._rc(rc)
        return bool(ok.value)

    def time(self):
        t = ctypes.c_int64()
        self._rc(self.lib.nphase_lbm_time(self.h, ctypes.byref(t)))
        return t.value

    def state_bytes(self):
        n = ctypes.c_size_t()
        self._rc(self.lib.nphase_lbm_state_bytes(self.h, ctypes.byref(n)))
        return n.value

    def save_state(self, buf=None):
        t = self.torch
        if buf is None:
            buf = t.empty(self.state_bytes(), dtype=t.uint8, device=self.device)
        self._rc(self.lib.nphase_lbm_save_state(self.h, ctypes.c_void_p(buf.data_ptr())))
        return buf

    def load_state(self, buf):
        self._rc(self.lib.nphase_lbm_load_state(self.h, ctypes.c_void_p(buf.data_ptr())))
        return self

    def state64_bytes(self):
        n = ctypes.c_size_t()
        self._rc(self.lib.nphase_lbm_state64_bytes(self.h, ctypes.byref(n)))
        return n.value

    def save_state64(self, buf=None):
        """The state as FP64 populations (the layout the adjoint reads)."""
        t = self.torch
        if buf is None:
            buf = t.empty(self.state64_bytes(), dtype=t.uint8, device=self.device)
        self._rc(self.lib.nphase_lbm_save_state64(self.h, ctypes.c_void_p(buf.data_ptr())))
        return buf

    # ---- discrete adjoint (FP64 arithmetic; state buffers in the save_state64 layout) -----
    def adjoint_workspace(self):
        n = ctypes.c_size_t()
        self._rc(self.lib.nphase_lbm_adjoint_workspace_bytes(self.h, ctypes.byref(n)))
        t = self.torch
        return t.empty(n.value + 256, dtype=t.uint8, device=self.device), n.value

    def adjoint_seed(self, dL_dphi, buf=None):
        t = self.torch
        x = dL_dphi.to(device=self.device, dtype=t.float64).contiguous()
        if buf is None:
            buf = t.zeros(self.state64_bytes(), dtype=t.uint8, device=self.device)
        self._rc(self.lib.nphase_lbm_adjoint_seed(self.h, ctypes.c_void_p(x.data_ptr()),
                                                  ctypes.c_void_p(buf.data_ptr())))
        return buf

    def adjoint_step(self, state_buf, lam_in, lam_out, ws):
        buf, nbytes = ws
        base = (buf.data_ptr() + 255) // 256 * 256
        self._rc(self.lib.nphase_lbm_adjoint_step(
            self.h, ctypes.c_void_p(state_buf.data_ptr()), ctypes.c_void_p(lam_in.data_ptr()),
            ctypes.c_void_p(lam_out.data_ptr()), ctypes.c_void_p(base), nbytes))
        return lam_out

    def adjoint_sigma(self, ws, reset=False, read=True):
        """dL/dsigma as an N x N matrix (pair derivative in both [p][q] and [q][p])."""
        buf, nbytes = ws
        base = (buf.data_ptr() + 255) // 256 * 256
        out = (ctypes.c_double * (MAX_N * MAX_N))()
        self._rc(self.lib.nphase_lbm_adjoint_sigma(self.h, ctypes.c_void_p(base),
                                                   out if read else None, 1 if reset else 0))
        if not read:
            return None
        m = np.array(out[:], dtype=np.float64).reshape(MAX_N, MAX_N)
        return m[:self.N, :self.N].copy()

    def adjoint_init(self, lam, ws):
        """dL/dphi0 from the adjoint of the initial state and the rho_bar partials in ws."""
        t = self.torch
        buf, nbytes = ws
        base = (buf.data_ptr() + 255) // 256 * 256
        out = t.empty((self.N,) + self.grid, dtype=t.float64, device=self.device)
        self._rc(self.lib.nphase_lbm_adjoint_init(self.h, ctypes.c_void_p(lam.data_ptr()),
                                                  ctypes.c_void_p(base), nbytes,
                                                  ctypes.c_void_p(out.data_ptr())))
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.nphase_lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
