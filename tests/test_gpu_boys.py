"""The device Boys function on its own (both forms the integral kernels use,
FP64 and FP32), against the oracle's F_j(T), which is pinned to the
incomplete gamma function through mpmath.

Arguments cover the table grid T_k = k/16 and the points halfway between
(the largest Taylor step), T -> 0, the FP32 form's switches at 1e-3 and 30,
the large-T switch at 60 and far beyond, plus a seeded uniform sample.
Bars: FP64 within 1e-14 relative for every order 0..8; FP32 within 2e-6
relative of F_j at the FP32-rounded argument where F_j >= 1e-30 (below, FP32
underflows and only |F| < 1e-29 is asked).
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

M = 8


def _arguments():
    grid = np.arange(0, 961, 7) / 16.0
    half = (np.arange(0, 960, 5) + 0.5) / 16.0
    special = [0.0, 1e-300, 1e-14, 1e-8, 1e-4, 9.999e-4, 1e-3, 1.0001e-3, 0.5, 29.999, 30.0, 30.001,
               59.96875, 59.999999, 60.0, 60.000001, 61.0, 80.0, 500.0, 1e6]
    rng = np.random.Generator(np.random.PCG64(17))
    return np.concatenate([grid, half, special, rng.uniform(0.0, 70.0, 400)])


@pytest.fixture(scope="module")
def basis():
    mess = need_gpu()
    B = mess.basis_from_molecule(G.random_small_molecule(1))
    yield B
    B.close()


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_boys_against_oracle(basis, form, prec):
    mess = need_gpu()
    torch = pytest.importorskip("torch")
    T = _arguments()
    Td = dev(T)
    F = torch.zeros(len(T), M + 1, dtype=torch.float64, device="cuda")
    p = mess.MESS_FP32 if prec == "fp32" else mess.MESS_FP64
    announce(f"boys form {form} {prec}: {len(T)} arguments, orders 0..{M}")
    mess.mess_boys(basis, Td, F, M, form=form, prec=p)
    got = host(F)
    Tref = T.astype(np.float32).astype(np.float64) if prec == "fp32" else T
    ref = np.array([core.boys(M, float(t)) for t in Tref])
    rel = np.abs(got - ref) / np.abs(ref)
    if prec == "fp32":
        # F_j below 1e-30 (orders 5..8 far out in T) leaves FP32's normal
        # range: there only the magnitude is checked
        tiny = ref < 1e-30
        assert np.all(np.abs(got[tiny]) < 1e-29)
        rel[tiny] = 0.0
    i, j = np.unravel_index(np.argmax(rel), rel.shape)
    announce(f"  worst relative error {rel.max():.2e} at T = {Tref[i]!r}, order {j}")
    assert rel.max() <= (2e-6 if prec == "fp32" else 1e-14)


def test_boys_lower_orders_and_edges(basis):
    mess = need_gpu()
    torch = pytest.importorskip("torch")
    T = np.array([0.0, 2.25, 45.0])
    # the recursion form computes F_0..F_m for the m asked for: each m agrees
    for m in range(M + 1):
        F = torch.zeros(len(T), m + 1, dtype=torch.float64, device="cuda")
        mess.mess_boys(basis, dev(T), F, m)
        ref = np.array([core.boys(m, float(t)) for t in T])
        assert np.max(np.abs(host(F) - ref) / ref) <= 1e-14
    # F_j(0) = 1/(2j+1), to the last bit
    F = torch.zeros(1, M + 1, dtype=torch.float64, device="cuda")
    mess.mess_boys(basis, dev(np.zeros(1)), F, M)
    exact = 1.0 / (2 * np.arange(M + 1) + 1)
    assert np.all(np.abs(host(F)[0] - exact) <= np.spacing(exact))
    # a negative argument gives NaN, not a table read
    F = torch.zeros(2, M + 1, dtype=torch.float64, device="cuda")
    mess.mess_boys(basis, dev(np.array([-1.0, 1.0])), F, M)
    h = host(F)
    assert np.all(np.isnan(h[0])) and np.all(np.isfinite(h[1]))
    # orders beyond the tables are refused
    with pytest.raises(mess.MessError):
        mess.mess_boys(basis, dev(T), torch.zeros(3, 10, dtype=torch.float64, device="cuda"), 9)
