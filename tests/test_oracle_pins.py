"""Pins of the CPU oracle against closed forms, brute force and invariants.

None of these re-types the oracle's own formulas: Boys values come from the
incomplete gamma function at 40 digits, integrals from direct numerical
quadrature of their definitions, energies from textbook closed forms of
one-Gaussian systems, and the rest from symmetries the exact answer has.
"""
import math
import os
import sys

import mpmath
import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import closed_forms as CF  # noqa: E402
import quadrature as Q  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import core, scf  # noqa: E402

mpmath.mp.dps = 40


def boys_mp(n, T):
    if T == 0:
        return mpmath.mpf(1) / (2 * n + 1)
    T = mpmath.mpf(T)
    return mpmath.gammainc(n + mpmath.mpf(1) / 2, 0, T) / (2 * T ** (n + mpmath.mpf(1) / 2))


# ---------------------------------------------------------------- Boys

@pytest.mark.parametrize("T", [0.0, 1e-14, 1e-6, 1e-3, 0.1, 0.5, 1.0, 3.7, 9.99, 15.0,
                               19.999, 20.0, 20.001, 25.0, 30.0, 36.0, 45.0, 80.0, 500.0])
def test_boys_matches_incomplete_gamma(T):
    F = core.boys(16, T)
    for n in range(17):
        ref = float(boys_mp(n, T))
        assert abs(F[n] - ref) <= 2e-15 * abs(ref), (n, T, F[n], ref)


def test_boys_special_values_and_recurrence():
    F0 = core.boys(16, 0.0)
    assert np.allclose(F0, [1.0 / (2 * n + 1) for n in range(17)], rtol=0, atol=0)
    # downward recurrence F_n = (2T F_{n+1} + e^-T)/(2n+1) holds at any T
    for T in [0.3, 7.0, 21.0, 44.0]:
        F = core.boys(12, T)
        for n in range(12):
            assert abs(F[n] - (2 * T * F[n + 1] + math.exp(-T)) / (2 * n + 1)) <= 2e-15 * F[n]
    # printed 40-digit reference values
    assert abs(core.boys(0, 1.0)[0] - 0.7468241328124270254) < 4e-16
    assert abs(core.boys(8, 30.0)[8] - 1.9526884564350918265e-9) < 1e-24


# ------------------------------------------------------ one-electron

def _tiny_spd(seed=3, n_atoms=3, alpha=(0.3, 3.0)):
    """A few atoms carrying single-primitive s, p, d shells (quadrature-friendly)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz = rng.uniform(0, 2.5, size=(n_atoms, 3))
    shells = []
    for a in range(n_atoms):
        for l in (0, 1, 2):
            shells.append((a, l, np.exp(rng.uniform(np.log(alpha[0]), np.log(alpha[1]), 1)),
                           np.array([1.0])))
    return G._assemble([1, 1, 2][:n_atoms], xyz, shells, "tiny_spd")


def test_unit_self_overlap_and_overlap_by_quadrature():
    for mol in (G.random_small_molecule(0), G.water_cluster(0, n_waters=1, box=4.0)):
        S, _, _ = core.one_electron(mol)
        assert np.max(np.abs(np.diag(S) - 1.0)) < 1e-14
        f = Q.basis_functions(mol, core.coefficients(mol))
        rng = np.random.Generator(np.random.PCG64(1))
        for i, j in list(zip(rng.integers(0, mol.n_bf, 25), rng.integers(0, mol.n_bf, 25))) + [(0, 0)]:
            ref = Q.overlap(f[i], f[j])
            assert abs(S[i, j] - ref) < 1e-13, (i, j)
        for i in range(mol.n_bf):           # unit self-overlap by quadrature, every component
            assert abs(Q.overlap(f[i], f[i]) - 1.0) < 1e-13


def _contracted_shells(seed=11):
    """Shells of 3-6 primitives with raw contraction coefficients drawn as
    the workloads draw them (exponents log-uniform in [0.05, 5000],
    coefficients uniform in (0, 1]), one s, p and d shell per atom."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz = rng.uniform(0, 2.0, size=(2, 3))
    shells = []
    for a in range(2):
        for l in (0, 1, 2):
            k = int(rng.integers(3, 7))
            shells.append((a, l, np.exp(rng.uniform(np.log(0.05), np.log(5000.0), k)),
                           1.0 - rng.uniform(0.0, 1.0, k)))
    return G._assemble([8, 1], xyz, shells, "contracted_spd")


def test_contraction_weights_from_raw_coefficients():
    """Reading of the contraction coefficients: each raw coefficient
    multiplies a primitive normalised to unit self-overlap, and the sum is
    renormalised.  Built here from the raw (exponent, coefficient) lists with
    every norm taken by quadrature of the squared function, so a weighting
    of raw primitives or a wrong primitive norm fails."""
    mol = _contracted_shells()
    got = core.coefficients(mol)
    p0 = 0
    for s in range(mol.n_shells):
        l, k = int(mol.shell_l[s]), int(mol.shell_nprim[s])
        ex, raw = mol.exps[p0:p0 + k], mol.coefs[p0:p0 + k]
        for c, lmn in enumerate(Q.cart_components(l)):
            def ov(a, b):
                return np.prod([Q.overlap_1d(lmn[x], 0.0, a, lmn[x], 0.0, b) for x in range(3)])
            nprim = np.array([1.0 / math.sqrt(ov(a, a)) for a in ex])
            w = raw * nprim
            self_ov = sum(w[i] * w[j] * ov(ex[i], ex[j]) for i in range(k) for j in range(k))
            want = w / math.sqrt(self_ov)
            assert np.max(np.abs(got[p0:p0 + k, c] - want) / np.abs(want)) < 1e-13, (s, c)
            # the raw-primitive weighting differs from the reading by far more
            wraw = raw / math.sqrt(sum(raw[i] * raw[j] * ov(ex[i], ex[j]) for i in range(k) for j in range(k)))
            assert np.max(np.abs(wraw - want) / np.abs(want)) > 1e-3
        p0 += k


def test_kinetic_and_nuclear_by_quadrature():
    mol = _tiny_spd()
    S, T, V = core.one_electron(mol)
    f = Q.basis_functions(mol, core.coefficients(mol))
    N = mol.n_bf
    rng = np.random.Generator(np.random.PCG64(2))
    pairs = [(i, j) for i, j in zip(rng.integers(0, N, 12), rng.integers(0, N, 12))]
    for i, j in pairs:
        assert abs(T[i, j] - Q.kinetic(f[i], f[j])) < 1e-12
        vref = sum(Q.nuclear(f[i], f[j], mol.xyz[c], mol.Z[c]) for c in range(mol.n_atoms))
        assert abs(V[i, j] - vref) < 1e-10 * max(1.0, abs(vref)), (i, j, V[i, j], vref)


def test_s_primitive_closed_forms():
    for alpha in (0.1, 1.0, 7.3):
        mol = G.single_gaussian_system("H", alpha)
        S, T, V = core.one_electron(mol)
        assert abs(T[0, 0] - 1.5 * alpha) < 1e-14 * max(1, alpha)
        assert abs(V[0, 0] + 2.0 * math.sqrt(2 * alpha / math.pi)) < 1e-14
        assert abs(core.eri_dense(mol)[0, 0, 0, 0] - 2.0 * math.sqrt(alpha / math.pi)) < 1e-15
    # one-electron H atom: E(alpha) = 3a/2 - 2 sqrt(2a/pi) is minimised at a = 8/(9 pi)
    a_star = 8.0 / (9.0 * math.pi)
    e = lambda a: float(np.sum(core.one_electron(G.single_gaussian_system("H", a))[1:]))  # noqa: E731
    assert abs(e(a_star) + 4.0 / (3.0 * math.pi)) < 1e-14
    assert e(a_star * 1.01) > e(a_star) and e(a_star * 0.99) > e(a_star)


# ------------------------------------------------------------- ERIs

def _ss_closed_form(a, A, b, B, c, C, d, D):
    return CF.ss_eri(a, A, b, B, c, C, d, D)


def test_ssss_analytic():
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(20):
        ex = np.exp(rng.uniform(np.log(0.05), np.log(500.0), 4))
        xyz = rng.uniform(-2, 2, size=(4, 3))
        shells = [(k, 0, ex[k:k + 1], np.array([1.0])) for k in range(4)]
        mol = G._assemble([1, 1, 1, 1], xyz, shells, "ssss")
        v = core.eri_shell_quartet(mol, 0, 1, 2, 3)[0, 0, 0, 0]
        ref = _ss_closed_form(ex[0], xyz[0], ex[1], xyz[1], ex[2], xyz[2], ex[3], xyz[3])
        assert abs(v - ref) <= 1e-14 * abs(ref) + 1e-16


@pytest.mark.parametrize("quartet", [(1, 0, 0, 0), (2, 0, 3, 0), (1, 4, 2, 7), (2, 5, 8, 4),
                                     (5, 8, 2, 5), (8, 8, 8, 8), (2, 2, 5, 1)])
def test_eri_against_gauss_transform_quadrature(quartet):
    mol = _tiny_spd()
    f = Q.basis_functions(mol, core.coefficients(mol))
    a, b, c, d = quartet
    blk = core.eri_shell_quartet(mol, a, b, c, d)
    bf0 = mol.bf_offsets()
    rng = np.random.Generator(np.random.PCG64(sum(quartet)))
    for _ in range(3):
        idx = [int(rng.integers(0, s)) for s in blk.shape]
        ref = Q.eri(*(f[bf0[sh] + i] for sh, i in zip(quartet, idx)))
        assert abs(blk[tuple(idx)] - ref) <= 1e-11 * max(1.0, abs(ref)), (quartet, idx)


def test_eri_eightfold_symmetry_and_schwarz():
    mol = G.random_small_molecule(1)
    E = core.eri_dense(mol)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 0, 1),
                 (2, 3, 1, 0), (3, 2, 1, 0)]:
        assert np.max(np.abs(E - E.transpose(perm))) < 1e-13 * np.max(np.abs(E))
    N = mol.n_bf
    M = E.reshape(N * N, N * N)
    diag = np.diag(M)
    assert np.all(np.abs(M) <= np.sqrt(np.outer(diag, diag)) * (1 + 1e-12) + 1e-14)
    w = np.linalg.eigvalsh(M)
    assert w.min() > -1e-12 * w.max()
    # shell-level Schwarz factors bound every block
    Qs = core.schwarz(mol)
    bf0, l = mol.bf_offsets(), mol.shell_l
    for a in range(mol.n_shells):
        for b in range(mol.n_shells):
            blk = E[bf0[a]:bf0[a] + core.ncart(l[a]), bf0[b]:bf0[b] + core.ncart(l[b]),
                    bf0[a]:bf0[a] + core.ncart(l[a]), bf0[b]:bf0[b] + core.ncart(l[b])]
            n = blk.shape[0] * blk.shape[1]
            assert abs(Qs[a, b] - math.sqrt(np.max(np.abs(np.diag(blk.reshape(n, n)))))) < 1e-15


def test_eri_translation_rotation_invariance():
    mol = G.random_small_molecule(2)
    moved = mol.copy()
    rng = np.random.Generator(np.random.PCG64(9))
    R = G._random_rotation(rng)
    moved.xyz = mol.xyz @ R.T + rng.normal(size=3)
    # s-only and full contractions with a rotation-invariant density give equal traces
    e1, e2 = core.eri_dense(mol), core.eri_dense(moved)
    ss = [i for i, l in enumerate(np.repeat(mol.shell_l, [core.ncart(x) for x in mol.shell_l])) if l == 0]
    sub = np.ix_(ss, ss, ss, ss)
    assert np.max(np.abs(e1[sub] - e2[sub])) < 1e-12


# ------------------------------------------------------------- J / K

def test_jk_digestion_rule_matches_definition():
    for mol in (G.random_small_molecule(0), _tiny_spd(seed=4)):
        N = mol.n_bf
        rng = np.random.Generator(np.random.PCG64(3))
        A = rng.normal(size=(N, N))
        D = A + A.T
        Jd, Kd = core.jk_from_dense(core.eri_dense(mol), D)
        Ju, Ku, n = core.jk_unique(mol, D, 0.0)
        npair = mol.n_shells * (mol.n_shells + 1) // 2
        assert n == npair * (npair + 1) // 2
        assert np.max(np.abs(Ju - Jd)) < 1e-12 * np.max(np.abs(Jd))
        assert np.max(np.abs(Ku - Kd)) < 1e-12 * np.max(np.abs(Kd))
        mu, nu = rng.integers(0, N, 6), rng.integers(0, N, 6)
        Je, Ke = core.jk_elements(mol, D, mu, nu)
        assert np.max(np.abs(Je - Jd[mu, nu])) < 1e-12 * np.max(np.abs(Jd))
        assert np.max(np.abs(Ke - Kd[mu, nu])) < 1e-12 * np.max(np.abs(Kd))
        # screening at a tiny threshold changes nothing visible
        Js, Ks, ns = core.jk_unique(mol, D, 1e-14)
        assert ns <= n and np.max(np.abs(Js - Jd)) < 1e-10


# ------------------------------------------------------------- SCF

def test_he_single_gaussian_rhf():
    k = (8 * math.sqrt(2) - 2) / math.sqrt(math.pi)
    for alpha in (0.4, 0.7669956643818522, 1.3):
        r = scf.RHF(G.single_gaussian_system("He", alpha)).run()
        assert abs(r["energy"] - (3 * alpha - k * math.sqrt(alpha))) < 1e-13
    a_star = (k / 6.0) ** 2
    assert abs(a_star - 0.7669956643818522) < 1e-15
    r = scf.RHF(G.single_gaussian_system("He", a_star)).run()
    assert abs(r["energy"] + k * k / 12.0) < 1e-13


def test_h2_minimal_basis_closed_form():
    for alpha, R in ((0.5, 1.4), (0.27, 2.0), (1.1, 0.9)):
        E_ref = CF.h2_minimal_energy(alpha, R)
        r = scf.RHF(G.single_gaussian_system("H2", alpha, bond=R)).run()
        assert abs(r["energy"] - E_ref) < 1e-13, (alpha, R, r["energy"], E_ref)
    assert abs(CF.h2_minimal_energy(0.5, 1.4) - (-0.9552136651016611)) < 1e-15


def test_converged_scf_invariants_and_invariance():
    mol = G.random_small_molecule(1)
    rhf = scf.RHF(mol, conv_tol=1e-12, max_iter=200)
    r = rhf.run()
    assert r["converged"]
    D, F, S = r["D"], r["F"], rhf.S
    assert np.max(np.abs(D @ S @ D - 2 * D)) < 1e-10          # idempotency
    assert np.max(np.abs(rhf.commutator(F, D))) < 1e-5       # Roothaan stationarity
    _, C, eps = scf.density_from_fock(F, rhf.X, rhf.n_occ)
    assert np.max(np.abs(C.T @ S @ C - np.eye(C.shape[1]))) < 1e-10   # eq. 5
    # E = E_elec + E_nuc
    J, K = rhf.jk(D)
    e_elec = 0.5 * np.sum(D * (2 * rhf.H + J - 0.5 * K))
    assert abs(r["energy"] - (e_elec + rhf.e_nuc)) < 1e-10
    # rigid motion of the molecule leaves the energy unchanged
    moved = mol.copy()
    rng = np.random.Generator(np.random.PCG64(4))
    moved.xyz = mol.xyz @ G._random_rotation(rng).T + rng.normal(size=3) * 3
    r2 = scf.RHF(moved, conv_tol=1e-12, max_iter=200).run()
    assert abs(r2["energy"] - r["energy"]) < 1e-9


def test_dense_and_unique_scf_agree():
    mol = G.random_small_molecule(3)
    r1 = scf.RHF(mol, jk="dense").run()
    r2 = scf.RHF(mol, jk="unique", tau=1e-12).run()
    assert abs(r1["energy"] - r2["energy"]) < 1e-9
