"""Mixed-precision path: FP32 primitive ERIs and FP32 J/K partial sums
(FP64 Boys near T = 0 and at large T, FP64 eigen-problem and energy).

The errors are stated against the FP64 oracle.  Bounds: J/K built in FP32
from a converged density stay within 2e-5 of the largest element; the FP32
SCF (incremental dD builds in FP32, full builds in FP64) reaches the oracle's
converged energy to 1e-6 Ha.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import announce, dev, host, need_gpu, zeros  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import core  # noqa: E402
from oracle import scf as oscf  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = {
    "hco6_sp/1": lambda: G.random_small_molecule(1),
    "water2_spd/0": lambda: G.water_cluster(0, n_waters=2, box=7.0),
    "mol3to20/1003": lambda: G.batched_molecule(1003),
}


@pytest.mark.parametrize("case", list(CASES))
def test_fp32_jk_error_at_converged_density(case):
    mess = need_gpu()
    mol = CASES[case]()
    ref = oscf.RHF(mol, conv_tol=1e-10, max_iter=200).run()
    D = ref["D"]
    Jo, Ko = core.jk_from_dense(core.eri_dense(mol), D)
    B = mess.basis_from_molecule(mol)
    N = B.nbf
    J, K = zeros(N, N), zeros(N, N)
    mess.mess_jk(B, dev(D), J, K, prec=mess.MESS_FP32, schwarz_tol=0.0)
    dJ = np.max(np.abs(host(J) - Jo)) / np.max(np.abs(Jo))
    dK = np.max(np.abs(host(K) - Ko)) / np.max(np.abs(Ko))
    announce(f"fp32 jk {case}: max|dJ|/max|J| = {dJ:.2e}, max|dK|/max|K| = {dK:.2e}")
    assert dJ < 2e-5 and dK < 2e-5


@pytest.mark.parametrize("case", list(CASES))
def test_fp32_scf_energy(case):
    mess = need_gpu()
    mol = CASES[case]()
    ref = oscf.RHF(mol, conv_tol=1e-10, max_iter=200).run()
    B = mess.basis_from_molecule(mol)
    st = mess.mess_scf_create(B, schwarz_tol=0.0, conv_tol=1e-9, diis_size=8, prec=mess.MESS_FP32)
    for _ in range(200):
        e, de, resid, conv = mess.mess_scf_step(st)
        if conv:
            break
    announce(f"fp32 scf {case}: E = {e:.10f}, oracle {ref['energy']:.10f}, |dE| = {abs(e - ref['energy']):.2e}")
    assert conv
    assert abs(e - ref["energy"]) < 1e-6


def test_fp32_eri_dense_error():
    mess = need_gpu()
    mol = G.water_cluster(0, n_waters=2, box=7.0)
    B = mess.basis_from_molecule(mol)
    N = B.nbf
    out = zeros(N, N, N, N)
    mess.mess_eri(B, out, prec=mess.MESS_FP32, schwarz_tol=0.0)
    ref = core.eri_dense(mol)
    err = np.max(np.abs(host(out) - ref) / np.maximum(1.0, np.abs(ref)))
    announce(f"fp32 eri water2: max |d|/max(1,|x|) = {err:.2e}")
    assert err < 1e-4
