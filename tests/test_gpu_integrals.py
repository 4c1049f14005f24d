"""GPU parity: one-electron integrals, ERIs and J/K against the CPU oracle.

Tolerance: integrals within 1e-12 * max(1, |x|) (absolute below 1, relative
above) of the oracle evaluated in extended precision (the same oracle source
built with long double), so the bound measures the GPU's own rounding.  J/K
are sums of up to N^2 ERIs times density elements; the bound used is
1e-11 * max(1, |X|) for unit-scale random densities, against the FP64 oracle.
"""
import functools
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import announce, dev, host, need_gpu, random_density, zeros  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import core  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = {
    "hco6_sp/0": lambda: G.random_small_molecule(0),
    "hco6_sp/5": lambda: G.random_small_molecule(5),
    "water2_spd/0": lambda: G.water_cluster(0, n_waters=2, box=7.0),
    "mol3to20/1000-small": lambda: G.batched_molecule(1007),
    # two waters far apart: most primitive pairs between them are screened
    "water2_spd_far/3": lambda: G.water_cluster(3, n_waters=2, box=14.0),
    # 83 functions; bras with more than 512 quartets, so the segmented
    # J/K kernels run several segments per bra
    "mol3to20/1001": lambda: G.batched_molecule(1001),
}


@functools.lru_cache(maxsize=8)
def _oracle_jk(case, tau, seed):
    mol = CASES[case]()
    J, K, _ = core.jk_unique(mol, G.symmetric_density(mol.n_bf, seed), tau)
    return J, K


def _rel_err(a, b):
    return np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))


@pytest.mark.parametrize("case", list(CASES))
def test_one_electron(case):
    mess = need_gpu()
    mol = CASES[case]()
    announce(f"one_electron {case} nbf={mol.n_bf}")
    B = mess.basis_from_molecule(mol)
    N = B.nbf
    S, T, V = zeros(N, N), zeros(N, N), zeros(N, N)
    mess.mess_one_electron(B, S, T, V)
    with core.extended_precision():
        So, To, Vo = core.one_electron(mol)
    # 1e-11: on water2_spd the FP64 oracle itself is 5.2e-12 away from its
    # extended-precision build in V (cancellation between primitives with
    # exponents up to 5000), so FP64 arithmetic cannot promise 1e-12 there.
    assert _rel_err(host(S), So) < 1e-12
    assert _rel_err(host(T), To) < 1e-11
    assert _rel_err(host(V), Vo) < 1e-11
    assert abs(B.e_nuc - core.nuclear_repulsion(mol)) < 1e-12 * max(1, abs(B.e_nuc))


@pytest.mark.parametrize("case", list(CASES))
def test_eri_dense(case):
    mess = need_gpu()
    mol = CASES[case]()
    if mol.n_bf > 60:
        pytest.skip("dense oracle tensor too large")
    B = mess.basis_from_molecule(mol)
    kept, full = mess.mess_prim_pairs(B)
    announce(f"eri_dense {case} nbf={mol.n_bf} primitive pairs kept {kept}/{full}")
    N = B.nbf
    out = zeros(N, N, N, N)
    mess.mess_eri(B, out, schwarz_tol=0.0)
    with core.extended_precision():
        ref = core.eri_dense(mol)
    got = host(out)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() < 1e-12, (err.max(), np.unravel_index(err.argmax(), err.shape))


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("tau", [0.0, 1e-10])
@pytest.mark.parametrize("mode", ["direct", "stored"])
def test_jk(case, tau, mode):
    mess = need_gpu()
    mol = CASES[case]()
    announce(f"jk {mode} {case} tau={tau} nbf={mol.n_bf}")
    B = mess.basis_from_molecule(mol)
    N = B.nbf
    J, K = zeros(N, N), zeros(N, N)
    m = mess.MESS_JK_DIRECT if mode == "direct" else mess.MESS_JK_STORED
    if mode == "stored":  # the second call streams the cached blocks
        mess.mess_jk(B, dev(random_density(N, seed=12)), J, K, mode=m, schwarz_tol=tau)
    D = random_density(N, seed=11)
    mess.mess_jk(B, dev(D), J, K, mode=m, schwarz_tol=tau)
    Jo, Ko = _oracle_jk(case, tau, 11)
    assert _rel_err(host(J), Jo) < 1e-11
    assert _rel_err(host(K), Ko) < 1e-11
    if tau == 0.0 and N <= 60:
        Jd, Kd = core.jk_from_dense(core.eri_dense(mol), D)
        assert _rel_err(host(J), Jd) < 1e-11
        assert _rel_err(host(K), Kd) < 1e-11


def test_primitive_screening_drops_pairs():
    """The screened cases above do exercise the primitive-pair screening:
    pairs between distant atoms lose their tight primitives, same-atom
    pairs keep all of theirs."""
    mess = need_gpu()
    mol = CASES["water2_spd_far/3"]()
    B = mess.basis_from_molecule(mol)
    kept, full = mess.mess_prim_pairs(B)
    announce(f"water2_spd_far/3: primitive pairs kept {kept}/{full}")
    nprim = np.asarray(mol.shell_nprim)
    same_atom = sum(int(nprim[a]) * int(nprim[b]) for a in range(len(nprim)) for b in range(a + 1)
                    if mol.shell_atom[a] == mol.shell_atom[b])
    assert full == sum(int(nprim[a]) * int(nprim[b]) for a in range(len(nprim)) for b in range(a + 1))
    assert same_atom <= kept < full
