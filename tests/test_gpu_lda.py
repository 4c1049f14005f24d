"""GPU parity of LDA exchange (Dirac-Slater on the Becke molecular grid)
against the oracle: the grid point by point, rho at every point, E_x and
V_x, one LDA SCF step from the oracle's density, and the converged LDA SCF
energy.  At the 60-atom water cluster's full size: sampled grid points and
densities, and identities that hold at any size (electron count on the
grid, Tr[D V_x] = 4/3 E_x)."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import announce, dev, host, need_gpu, zeros  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import core as ocore  # noqa: E402
from oracle import lda as olda  # noqa: E402
from oracle import scf as oscf  # noqa: E402

pytestmark = pytest.mark.gpu


def _psd_density(n, nocc, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    C = rng.normal(size=(n, nocc)) / math.sqrt(n)
    return 2.0 * C @ C.T


def _check_weights(got, want, idx):
    """Weights = radial x angular x Becke factor.  The Becke factor (in
    [0, 1]) must agree to 1e-13 absolute: where it is tiny, s(mu) = (1 - f)/2
    with f near 1 cancels and only absolute accuracy is meaningful; the rule
    weights to 1e-11 relative: at the outermost radial node
    r = (1+x)/(1-x) with 1 - x ~ 1e-3 turns a one-ulp difference in cos(t)
    into ~1e-13 relative, grown further by r^2 / (1-x)^2."""
    r, wr = olda.radial_rule()
    _, wa = olda.angular_rule()
    rest = idx % (olda.N_RADIAL * len(wa))
    wra = wr[rest // len(wa)] * wa[rest % len(wa)]
    assert np.all(np.abs(got - want) <= 1e-11 * np.abs(want) + 1e-13 * wra)


def _gpu_grid(mess, B):
    n = mess.mess_grid(B)
    xyzw = zeros(n, 4)
    mess.mess_grid(B, xyzw)
    return host(xyzw)


@pytest.fixture(scope="module")
def small():
    mess = need_gpu()
    mol = G.random_small_molecule(1)
    announce(f"LDA small molecule nbf={mol.n_bf} atoms={len(mol.Z)}")
    return mess, mol, mess.basis_from_molecule(mol), olda.grid_points(mol)


def test_grid_matches_oracle(small):
    mess, mol, B, (pts, w) = small
    g = _gpu_grid(mess, B)
    assert g.shape == (olda.n_points(mol), 4)
    assert np.abs(g[:, :3] - pts).max() <= 1e-13 * max(1.0, np.abs(pts).max())
    _check_weights(g[:, 3], w, np.arange(len(w)))
    assert abs(g[:, 3].sum() - w.sum()) <= 1e-12 * w.sum()


def test_lda_x_matches_oracle(small):
    mess, mol, B, grid = small
    D = _psd_density(mol.n_bf, 10, 3)
    Ex_ref, V_ref, rho_ref = olda.lda_x(mol, D, grid=grid)
    V = zeros(mol.n_bf, mol.n_bf)
    rho = zeros(len(rho_ref))
    Ex = mess.mess_lda_x(B, dev(D), V, rho)
    assert abs(Ex - Ex_ref) <= 1e-11 * abs(Ex_ref), (Ex, Ex_ref)
    assert np.abs(host(rho) - rho_ref).max() <= 1e-12 * np.abs(rho_ref).max()
    Vh = host(V)
    assert np.abs(Vh - V_ref).max() <= 1e-11 * np.abs(V_ref).max()
    assert np.abs(Vh - Vh.T).max() == 0.0


def test_lda_scf_one_step_from_oracle_density(small):
    mess, mol, B, grid = small
    ref = oscf.RHF(mol, jk="dense", xc="lda")
    D = ref.core_guess()
    F_ref, E_ref = ref.fock(D)
    st = mess.mess_scf_create(B, schwarz_tol=0.0, diis_size=0, xc=mess.MESS_XC_LDA_X, D0=dev(D))
    e, de, r, c = mess.mess_scf_step(st)
    assert abs(e - E_ref) <= 1e-10 * abs(E_ref), (e, E_ref)
    F = zeros(mol.n_bf, mol.n_bf)
    mess.mess_scf_fock(st, F)
    assert np.abs(host(F) - F_ref).max() <= 1e-10 * np.abs(F_ref).max()


def test_lda_scf_converged_energy(small):
    mess, mol, B, grid = small
    ref = oscf.RHF(mol, jk="dense", xc="lda", conv_tol=1e-10, max_iter=100).run()
    assert ref["converged"]
    for mode in (mess.MESS_JK_DIRECT, mess.MESS_JK_STORED):
        st = mess.mess_scf_create(B, schwarz_tol=0.0, conv_tol=1e-10, diis_size=8, xc=mess.MESS_XC_LDA_X,
                                  jk_mode=mode)
        for k in range(100):
            e, de, r, c = mess.mess_scf_step(st)
            if c:
                break
        assert c
        assert abs(e - ref["energy"]) < 1e-9, (mode, e, ref["energy"])


def test_lda_rejections(small):
    mess, mol, B, grid = small
    with pytest.raises(mess.MessError) as ei:
        mess.mess_scf_create(B, xc=mess.MESS_XC_LDA_X, prec=mess.MESS_FP32)
    assert ei.value.code == mess.MESS_E_UNSUPPORTED
    Bb = mess.mess_batch_create([mol, mol])
    with pytest.raises(mess.MessError) as ei:
        mess.mess_grid(Bb)
    assert ei.value.code == mess.MESS_E_UNSUPPORTED


def test_lda_full_size_water60():
    """60-atom water cluster (2.6e6 grid points, 300 functions): sampled
    grid points and densities against the oracle; electron count and the
    homogeneity identity Tr[D V_x] = 4/3 E_x over the whole grid."""
    mess = need_gpu()
    mol = G.water_cluster(0)
    announce(f"LDA water60 nbf={mol.n_bf}")
    B = mess.basis_from_molecule(mol)
    # the oracle's core-Hamiltonian guess density
    S, T, V = ocore.one_electron(mol)
    X = oscf.canonical_orthogonaliser(S)
    D = oscf.density_from_fock(T + V, X, mol.n_electrons // 2)[0]
    n = mess.mess_grid(B)
    assert n == olda.n_points(mol)
    g = _gpu_grid(mess, B)
    rng = np.random.Generator(np.random.PCG64(11))
    idx = np.sort(rng.choice(n, size=3000, replace=False))
    pts, w = olda.grid_points(mol, idx)
    assert np.abs(g[idx, :3] - pts).max() <= 1e-13 * max(1.0, np.abs(pts).max())
    _check_weights(g[idx, 3], w, idx)
    Vx = zeros(mol.n_bf, mol.n_bf)
    rho = zeros(n)
    Ex = mess.mess_lda_x(B, dev(D), Vx, rho)
    rh = host(rho)
    Phi = olda.basis_values(mol, pts)
    rho_ref = np.einsum("gm,mn,gn->g", Phi, D, Phi)
    assert np.abs(rh[idx] - rho_ref).max() <= 1e-11 * max(1.0, np.abs(rho_ref).max())
    # electrons on the grid (grid error with exponents up to 5000)
    assert abs(np.sum(g[:, 3] * rh) - mol.n_electrons) < 1e-3 * mol.n_electrons
    # E_x is homogeneous of degree 4/3 in rho, so sum D .* V_x = 4/3 E_x
    Vh = host(Vx)
    assert np.abs(Vh - Vh.T).max() == 0.0
    assert abs(np.sum(D * Vh) - 4.0 / 3.0 * Ex) <= 1e-10 * abs(Ex)
