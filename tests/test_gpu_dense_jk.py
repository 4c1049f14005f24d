"""GPU parity of the dense-tensor J/K contraction of many densities
(mess_jk_dense), both forms (matrix cores and vector FMAs), FP64 and FP32,
against the oracle's defining sums over its own dense ERI tensor.

Densities: 70 seeded symmetric matrices (a tile of 64 densities and a
ragged second one) on a 30-function molecule (900 composite indices: 14 row
tiles of 64 and a ragged last one).  Bars: FP64
within 1e-11 * max(1, |x|) (the GPU tensor itself is within 1e-12 of the
oracle's); FP32 within 2e-5 of max|J|, max|K|.  The two FP64 forms agree to
rounding (their sums differ only in order).
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import announce, dev, host, need_gpu  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import core  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    mess = need_gpu()
    torch = pytest.importorskip("torch")
    mol = G.random_small_molecule(2)
    N = mol.n_bf
    eri_o = core.eri_dense(mol)
    Ds = np.stack([G.symmetric_density(N, 60 + k) for k in range(70)])
    J = np.einsum("ijkl,dkl->dij", eri_o, Ds)
    K = np.einsum("ikjl,dkl->dij", eri_o, Ds)
    B = mess.basis_from_molecule(mol)
    eri64 = torch.zeros(N, N, N, N, dtype=torch.float64, device="cuda")
    mess.mess_eri(B, eri64, schwarz_tol=0.0)
    # the FP32 integral kernels write the dense tensor as doubles; the FP32
    # contraction takes it as floats
    e32 = torch.zeros(N, N, N, N, dtype=torch.float64, device="cuda")
    mess.mess_eri(B, e32, prec=mess.MESS_FP32, schwarz_tol=0.0)
    eri32 = e32.to(torch.float32)
    return mess, torch, N, Ds, J, K, eri64, eri32


@pytest.mark.parametrize("form", ["mfma", "valu"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dense_jk_matches_oracle(case, form, prec):
    mess, torch, N, Ds, Jo, Ko, eri64, eri32 = case
    f = mess.MESS_DENSE_MFMA if form == "mfma" else mess.MESS_DENSE_VALU
    dt = torch.float64 if prec == "fp64" else torch.float32
    p = mess.MESS_FP64 if prec == "fp64" else mess.MESS_FP32
    eri = eri64 if prec == "fp64" else eri32
    D = torch.tensor(Ds, dtype=dt, device="cuda")
    J = torch.zeros_like(D)
    K = torch.zeros_like(D)
    mess.mess_jk_dense(eri, N, D, J, K, prec=p, form=f)
    Jh, Kh = host(J).astype(np.float64), host(K).astype(np.float64)
    if prec == "fp64":
        eJ = np.max(np.abs(Jh - Jo) / np.maximum(1.0, np.abs(Jo)))
        eK = np.max(np.abs(Kh - Ko) / np.maximum(1.0, np.abs(Ko)))
        announce(f"dense jk {form} fp64: worst |d|/max(1,|x|) J {eJ:.1e} K {eK:.1e}")
        assert eJ < 1e-11 and eK < 1e-11
    else:
        eJ = np.max(np.abs(Jh - Jo)) / np.max(np.abs(Jo))
        eK = np.max(np.abs(Kh - Ko)) / np.max(np.abs(Ko))
        announce(f"dense jk {form} fp32: max|dJ|/max|J| {eJ:.1e}, max|dK|/max|K| {eK:.1e}")
        assert eJ < 2e-5 and eK < 2e-5


def test_dense_jk_forms_agree_and_edges(case):
    mess, torch, N, Ds, Jo, Ko, eri64, eri32 = case
    D = dev(Ds)
    out = {}
    for f in (mess.MESS_DENSE_MFMA, mess.MESS_DENSE_VALU):
        J, K = torch.zeros_like(D), torch.zeros_like(D)
        mess.mess_jk_dense(eri64, N, D, J, K, form=f)
        out[f] = (host(J), host(K))
    for a, b in zip(out[mess.MESS_DENSE_MFMA], out[mess.MESS_DENSE_VALU]):
        assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b)))
    # one density; J only
    J1 = torch.zeros(1, N, N, dtype=torch.float64, device="cuda")
    mess.mess_jk_dense(eri64, N, D[:1].contiguous(), J1, None)
    assert np.max(np.abs(host(J1)[0] - Jo[0])) <= 1e-11 * max(1.0, np.abs(Jo[0]).max())
    with pytest.raises(mess.MessError):
        mess.mess_jk_dense(eri64, N, D, J1, None, form=7)
