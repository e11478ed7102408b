"""The interface-location diagnostics without allocation (a handle-free C-ABI entry point
whose reduction scratch is a static device array of the library) against the handle's
entry point on the same fields: bitwise equal, on calls in a row on one GPU whose later
inputs are smaller (fewer phases, fewer nodes), so that nothing of an earlier call's
scratch contents leaks into a later result."""
import numpy as np
import pytest

from paper_2306_06983_amd import inputs

pytestmark = pytest.mark.gpu


def _fields(cfg, phi, steps=10):
    from paper_2306_06983_amd import binding as B
    s = B.Sim(cfg, "fp64").init(phi).step(steps)
    ph = s.fields()[0]
    return s, ph


def test_noalloc_locations_equal_handle_entry_point():
    from paper_2306_06983_amd import binding as B
    cases = [("D2Q9", inputs.many_discs(n=160, N=6, count=10, rmin=6, rmax=12)),
             ("D3Q19", inputs.spheres(n=32, scale=0.125)),
             ("D2Q9", inputs.two_discs())]
    sizes = []
    for lattice, (cfg, phi) in cases:
        s, ph = _fields(cfg, phi)
        want = s.interface_locations(ph)
        got = B.interface_locations_noalloc(ph, lattice)
        for w, g in zip(want, got):
            assert w.shape == g.shape == (cfg["n_phases"],)
            assert np.array_equal(w, g)
        present = got[1] >= 0
        assert np.all(got[2][present] >= got[1][present])
        assert np.all(got[2][~present] == -1)
        sizes.append((cfg["n_phases"], ph.numel()))
        s.close()
    # each call after the first has a smaller input than the one before it
    assert sizes[1][0] < sizes[0][0] and sizes[2][0] < sizes[1][0]
    assert sizes[2][1] < sizes[1][1] < sizes[0][1]


def test_noalloc_rejects_more_phases_than_the_scratch_holds():
    """More than NPHASE_MAX_N phases are refused on the host (ENOTSUP, no device work);
    bad extents with EINVAL."""
    import ctypes
    import torch
    from paper_2306_06983_amd import binding as B
    lib = B.load()
    phi = torch.zeros((9, 4, 4), dtype=torch.float64, device="cuda:0")
    av = (ctypes.c_double * 9)()
    lo = (ctypes.c_int32 * 9)()
    hi = (ctypes.c_int32 * 9)()
    rc = lib.nphase_lbm_interface_locations_noalloc(B.D2Q9, 4, 4, 1, 9,
                                                    ctypes.c_void_p(phi.data_ptr()), None,
                                                    av, lo, hi)
    assert rc == B.NPHASE_ENOTSUP
    rc = lib.nphase_lbm_interface_locations_noalloc(B.D2Q9, 4, 4, 2, 2,
                                                    ctypes.c_void_p(phi.data_ptr()), None,
                                                    av, lo, hi)
    assert rc == B.NPHASE_EINVAL
    # the entry point still works after the refusals
    cfg, ph0 = inputs.two_discs()
    s, ph = _fields(cfg, ph0, steps=3)
    for w, g in zip(s.interface_locations(ph), B.interface_locations_noalloc(ph, "D2Q9")):
        assert np.array_equal(w, g)
