"""CPU checks of the C-ABI library: it loads, exports every declared symbol, rejects bad
arguments before touching the GPU, and its host-side operator assembly matches the
oracle's matrices (no compute calls on a device)."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT
import paper_2506_14792_amd as sps
from paper_2506_14792_amd.sps import SpsDesc, make_desc
from oracle.rbc import RBC


def declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(sps_[A-Za-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = sps.lib()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n


def test_build_rejects_bad_arguments_without_gpu():
    L = sps.lib()
    h = ctypes.c_void_p()
    for d in (make_desc(sps.RBC2D, 255, 64, 4.0, 1e6, 1.0),             # odd nx
              make_desc(sps.RBC2D, 256, 130, 4.0, 1e6, 1.0),            # nz too large
              make_desc(sps.RBC2D, 256, 64, 4.0, 1e6, 1.0, scheme=sps.SBDF2),
              make_desc(sps.RBC2D, 256, 64, 4.0, 1e6, 1.0, dt=-1.0),
              make_desc(99, 256, 64)):
        rc = L.sps_build_problem(ctypes.byref(d), None, ctypes.byref(h))
        assert rc == -1 and not h.value
        assert len(L.sps_last_error()) > 0
    assert L.sps_sync(None) == -1


def reconstruct(hb, k, which):
    band = hb[which][k]
    S = band.shape[0]
    kl, ku = hb["kl"], hb["ku"]
    B = np.zeros((S, S))
    for i in range(S):
        for d in range(kl + ku + 1):
            j = i + d - kl
            if 0 <= j < S:
                B[i, j] = band[i, d]
    return B


@pytest.mark.parametrize("nx,nz,lx,Ra,Pr", [(16, 12, 3.0, 1e4, 0.7), (256, 64, 4.0, 1e6, 1.0)])
def test_host_bands_match_oracle_operators(nx, nz, lx, Ra, Pr):
    hb = sps.rbc_host_bands(nx, nz, lx, Ra, Pr)
    P = RBC(Nx=nx, Nz=nz, Lx=lx, Ra=Ra, Pr=Pr)
    S = P.S
    rowph = np.where(hb["rowph"] == 1, -1j, 1.0)
    colph = np.where(hb["colph"] == 1, 1j, 1.0)
    R = np.eye(S)
    for s in range(S - 2):
        R[s, s + 2] = hb["rho"][s]
    for k in sorted({0, 1, P.K // 2, P.K - 1}):
        for which, A in (("BM", P.M[k]), ("BL", P.L[k])):
            T = ((rowph[:, None] * A) @ R * colph[None, :])[np.ix_(hb["rowmap"], hb["colmap"])]
            assert np.abs(T.imag).max() <= 1e-13 * np.abs(T).max()
            B = reconstruct(hb, k, which)
            assert np.abs(T.real - B).max() <= 1e-14 * np.abs(T).max(), (k, which)
    if nz == 64:
        assert (hb["kl"], hb["ku"]) == (7, 20)


def test_set_allocator_arguments():
    """sps_set_allocator takes both functions or neither (no device needed)."""
    L = sps.lib()
    from paper_2506_14792_amd.sps import _ALLOC_T, _FREE_T
    fa = _ALLOC_T(lambda n, c: None)
    ff = _FREE_T(lambda p, c: None)
    a, f = ctypes.cast(fa, ctypes.c_void_p), ctypes.cast(ff, ctypes.c_void_p)
    assert L.sps_set_allocator(a, None, None) == -1
    assert L.sps_set_allocator(None, f, None) == -1
    assert L.sps_set_allocator(a, f, None) == 0
    assert L.sps_set_allocator(None, None, None) == 0
