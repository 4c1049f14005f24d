"""Every kernel form of every class (the choices the autotuner makes) meets
the same parity bar: with the form of one class forced, dense ERIs within
1e-12 * max(1, |x|) of the extended-precision oracle and direct J/K within
1e-11 * max(1, |x|) of the oracle's defining sums, for a molecule holding
every angular class.  FP32 table: with one class's FP32 form forced, FP32
J/K within 2e-5 of max|J|, max|K| (the FP32 bar of the mixed-precision
tests)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import announce, dev, host, need_gpu, random_density, zeros  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import core  # noqa: E402

pytestmark = pytest.mark.gpu

PC = ["ss", "ps", "pp", "ds", "dp", "dd"]
FORMS = {1: "lane", 2: "rows", 3: "plane", 4: "coop", 5: "wave", 6: "fp64"}


def _cases(forms, prec):
    """The (class, form) pairs the library has kernels for (the form table's
    validity check is host logic: no device needed to ask)."""
    out = [(cb, ck, f) for cb in range(6) for ck in range(cb + 1) for f in forms]
    try:
        from paper_2406_03121_amd import mess
        lib = mess.lib()
        p = mess.MESS_FP64 if prec == 64 else mess.MESS_FP32
    except Exception:  # library not built: every pair, each skipped at run time
        return out
    built = []
    for cb, ck, f in out:
        cls = cb * (cb + 1) // 2 + ck
        if lib.mess_kernel_form(p, cls, f, None) == mess.MESS_OK:
            built.append((cb, ck, f))
        lib.mess_kernel_form(p, cls, mess.MESS_FORM_AUTO, None)
    return built


@pytest.fixture(scope="module")
def ref():
    mol = G.water_cluster(0, n_waters=2, box=7.0)
    with core.extended_precision():
        eri = core.eri_dense(mol)
    D = random_density(mol.n_bf, seed=51)
    J, K = core.jk_from_dense(core.eri_dense(mol), D)
    return mol, eri, D, J, K


@pytest.mark.parametrize("cb,ck,form", _cases([1, 2, 3, 4, 5], 64))
def test_form_parity(ref, cb, ck, form):
    mess = need_gpu()
    cls = mess.class_index(cb, ck)
    if mess.lib().mess_kernel_form(mess.MESS_FP64, cls, form, None) != mess.MESS_OK:
        pytest.skip(f"form {FORMS[form]} not built for ({PC[cb]}|{PC[ck]})")
    try:
        mol, eri, D, Jo, Ko = ref
        announce(f"form {FORMS[form]} for ({PC[cb]}|{PC[ck]})")
        B = mess.basis_from_molecule(mol)
        N = B.nbf
        out = zeros(N, N, N, N)
        mess.mess_eri(B, out, schwarz_tol=0.0)
        got = host(out)
        err = np.abs(got - eri) / np.maximum(1.0, np.abs(eri))
        assert err.max() < 1e-12, err.max()
        for tau in (0.0, 1e-10):
            J, K = zeros(N, N), zeros(N, N)
            mess.mess_jk(B, dev(D), J, K, schwarz_tol=tau)
            if tau == 0.0:
                rel = lambda a, b: np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))  # noqa: E731
                assert rel(host(J), Jo) < 1e-11 and rel(host(K), Ko) < 1e-11
            else:
                Jt, Kt, _ = core.jk_unique(mol, D, tau)
                rel = lambda a, b: np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))  # noqa: E731
                assert rel(host(J), Jt) < 1e-11 and rel(host(K), Kt) < 1e-11
        B.close()
    finally:
        mess.mess_kernel_form(cls, mess.MESS_FORM_AUTO)


@pytest.mark.parametrize("cb,ck,form", _cases([1, 2, 3, 4, 5, 6], 32))
def test_fp32_form_parity(ref, cb, ck, form):
    mess = need_gpu()
    cls = mess.class_index(cb, ck)
    if mess.lib().mess_kernel_form(mess.MESS_FP32, cls, form, None) != mess.MESS_OK:
        pytest.skip(f"FP32 form {FORMS[form]} not built for ({PC[cb]}|{PC[ck]})")
    try:
        mol, eri, D, Jo, Ko = ref
        announce(f"fp32 form {FORMS[form]} for ({PC[cb]}|{PC[ck]})")
        B = mess.basis_from_molecule(mol)
        N = B.nbf
        J, K = zeros(N, N), zeros(N, N)
        mess.mess_jk(B, dev(D), J, K, prec=mess.MESS_FP32, schwarz_tol=0.0)
        dJ = np.max(np.abs(host(J) - Jo)) / np.max(np.abs(Jo))
        dK = np.max(np.abs(host(K) - Ko)) / np.max(np.abs(Ko))
        assert dJ < 2e-5 and dK < 2e-5, (dJ, dK)
        B.close()
    finally:
        mess.mess_kernel_form(cls, mess.MESS_FORM_AUTO, prec=mess.MESS_FP32)
