"""The allocation-free J/K entry point (mess_jk_noalloc) against mess_jk.

Called through the C ABI with ctypes.  Both run the same class kernels on
the same work lists; they differ only in where the half matrices live (a
fixed device array instead of the basis handle's buffer), so the results
agree to the order of the FP64 atomic additions.  Two calls in a row, the
second on a smaller molecule, check that the shared workspace is cleared
between calls.
"""
import ctypes
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import announce, dev, host, need_gpu, random_density, zeros  # noqa: E402

from mess_inputs import generators as G  # noqa: E402

pytestmark = pytest.mark.gpu


def _noalloc(mess):
    f = mess.lib().mess_jk_noalloc
    vp = ctypes.c_void_p
    f.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_double, vp]
    f.restype = ctypes.c_int
    return f


def _call(mess, f, B, D, J, K, tau, prec=0):
    p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())  # noqa: E731
    import torch
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return f(B.handle, p(D), p(J), p(K), int(prec), float(tau), stream)


def _rel(a, b):
    return np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))


@pytest.mark.parametrize("tau", [0.0, 1e-10])
def test_noalloc_matches_jk_twice(tau):
    mess = need_gpu()
    f = _noalloc(mess)
    cases = [("water3_spd/0", G.water_cluster(0, n_waters=3, box=8.0)),
             ("hco6_sp/5", G.random_small_molecule(5))]
    assert cases[1][1].n_bf < cases[0][1].n_bf
    for name, mol in cases:
        announce(f"noalloc jk {name} tau={tau} nbf={mol.n_bf}")
        B = mess.basis_from_molecule(mol)
        N = B.nbf
        D = dev(random_density(N, seed=31))
        J0, K0 = zeros(N, N), zeros(N, N)
        J1, K1 = zeros(N, N), zeros(N, N)
        # before the work lists exist the entry point refuses (it would allocate)
        assert _call(mess, f, B, D, J1, K1, tau) == mess.MESS_E_ARG
        assert "work lists" in mess.mess_last_error()
        mess.mess_jk(B, D, J0, K0, schwarz_tol=tau)
        assert _call(mess, f, B, D, J1, K1, tau) == mess.MESS_OK
        assert _rel(host(J1), host(J0)) < 1e-12
        assert _rel(host(K1), host(K0)) < 1e-12
        # J only, then K only
        J2, K2 = zeros(N, N), zeros(N, N)
        assert _call(mess, f, B, D, J2, None, tau) == mess.MESS_OK
        assert _call(mess, f, B, D, None, K2, tau) == mess.MESS_OK
        assert _rel(host(J2), host(J0)) < 1e-12
        assert _rel(host(K2), host(K0)) < 1e-12
        B.close()


def test_noalloc_rejects_oversized_and_fp32_matches():
    mess = need_gpu()
    f = _noalloc(mess)
    mol = G.random_small_molecule(2)
    B = mess.basis_from_molecule(mol)
    N = B.nbf
    D = dev(random_density(N, seed=32))
    J0, K0, J1, K1 = zeros(N, N), zeros(N, N), zeros(N, N), zeros(N, N)
    mess.mess_jk(B, D, J0, K0, prec=mess.MESS_FP32, schwarz_tol=0.0)
    assert _call(mess, f, B, D, J1, K1, 0.0, prec=mess.MESS_FP32) == mess.MESS_OK
    assert _rel(host(J1), host(J0)) < 1e-6
    assert _rel(host(K1), host(K0)) < 1e-6
    assert _call(mess, f, B, None, J1, K1, 0.0) == mess.MESS_E_ARG
    assert _call(mess, f, B, D, J1, K1, 0.0, prec=7) == mess.MESS_E_UNSUPPORTED
    B.close()
    # a batch whose packed matrices exceed the fixed workspace
    mols = G.batch_of_molecules(200)
    Bb = mess.mess_batch_create(mols)
    announce(f"noalloc oversized batch packed={Bb.packed}")
    assert Bb.packed > (1 << 19)
    Db = torch_zeros(Bb.packed)
    assert _call(mess, f, Bb, Db, None, None, 0.0) == mess.MESS_E_SIZE
    assert "workspace" in mess.mess_last_error()
    Bb.close()


def torch_zeros(n):
    import torch
    return torch.zeros(n, dtype=torch.float64, device="cuda")
