"""Pins of the learned-guess oracle (oracle/guess.py): BF16 rounding on known
bit patterns, the exact backward against central differences, Adam's
closed-form first step, feature invariances and special values, the block
round trip, and the projection's defining properties."""
import math

import numpy as np
import pytest

from mess_inputs import generators as G
from oracle import core, guess, scf


def test_bf16_rounding_known_values():
    one = 1.0
    cases = {
        one: one,
        one + 2 ** -8: one,                      # tie -> even (1.0)
        one + 3 * 2 ** -8: one + 2 ** -6,        # tie -> even (1 + 2^-6)
        one + 2 ** -8 + 2 ** -20: one + 2 ** -7,  # above the tie
        -(one + 2 ** -8 + 2 ** -20): -(one + 2 ** -7),
        3.0: 3.0,
        0.0: 0.0,
    }
    for x, want in cases.items():
        assert guess.bf16(np.array([x]))[0] == want, x
    # every BF16 value is a fixed point; results have 8 significant bits
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.normal(size=1000) * 10.0 ** rng.integers(-5, 5, size=1000)
    y = guess.bf16(x)
    assert np.array_equal(guess.bf16(y), y)
    assert np.all(np.abs(y - x) <= 2 ** -8 * np.abs(x))


def _batch(n=12, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.normal(size=(n, guess.N_IN))
    T = rng.normal(size=(n, guess.N_OUT)) * 0.1
    M = (rng.uniform(size=(n, guess.N_OUT)) < 0.6).astype(float)
    p = G.mlp_initial_params(3).astype(np.float64)
    p += rng.normal(size=p.shape) * 0.01  # non-zero biases too
    return p, X, T, M


def test_exact_backward_matches_central_differences():
    p, X, T, M = _batch()
    L, g = guess.loss_and_grad(p, X, T, M)
    rng = np.random.Generator(np.random.PCG64(2))
    offs = np.cumsum([0] + [int(np.prod(s)) for s in guess.SHAPES])
    for t in range(6):
        for k in rng.integers(offs[t], offs[t + 1], size=4):
            h = 1e-6
            pp, pm = p.copy(), p.copy()
            pp[k] += h
            pm[k] -= h
            fd = (guess.loss_and_grad(pp, X, T, M)[0] - guess.loss_and_grad(pm, X, T, M)[0]) / (2 * h)
            assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])), (t, k, fd, g[k])


def test_masked_entries_carry_no_gradient():
    p, X, T, M = _batch()
    T2 = T + (1.0 - M) * 5.0  # change only masked-out targets
    assert np.array_equal(guess.loss_and_grad(p, X, T, M)[1], guess.loss_and_grad(p, X, T2, M)[1])


def test_bf16_path_close_to_exact():
    p, X, T, M = _batch()
    Y, _ = guess.forward(p, X)
    Yb, _ = guess.forward_bf16(p, X)
    assert np.abs(Yb - Y).max() < 3e-2 * np.abs(Y).max()
    L, g = guess.loss_and_grad(p, X, T, M)
    Lb, gb = guess.loss_and_grad_bf16(p, X, T, M)
    assert abs(Lb - L) < 1e-2 * L
    assert np.abs(gb - g).max() < 5e-2 * np.abs(g).max()


def test_adam_first_step_closed_form():
    rng = np.random.Generator(np.random.PCG64(4))
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    p1, m, v = guess.adam(p, np.zeros(100), np.zeros(100), g, 1)
    # bias-corrected moments are g and g^2 after one step
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_feature_special_values_and_invariances():
    mol = G.batched_molecule(1000)
    F = guess.features(mol)
    P = guess.pairs(mol)
    assert F.shape == (len(P), 64) and len(P) == len(mol.Z) * (len(mol.Z) + 1) // 2
    assert np.all(F[:, 0:4].sum(1) == 1) and np.all(F[:, 4:8].sum(1) == 1)
    assert np.all(F[:, 42:] == 0)
    for r, (a, b) in enumerate(P):
        if a == b:
            assert F[r, 41] == 1 and np.all(F[r, 24:33] == 0) and F[r, 8] == 1.0
        else:
            assert F[r, 41] == 0 and abs(np.linalg.norm(F[r, 24:27]) - 1) < 1e-14
    # rigid motion: radial functions, counts and one-hots unchanged; u rotates
    rng = np.random.Generator(np.random.PCG64(5))
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    m2 = mol.copy()
    m2.xyz = (np.asarray(mol.xyz).reshape(-1, 3) @ Q.T + np.array([1.0, -2.0, 0.5])).ravel().reshape(
        np.asarray(mol.xyz).shape)
    F2 = guess.features(m2)
    keep = np.r_[0:24, 33:42]
    assert np.abs(F2[:, keep] - F[:, keep]).max() < 1e-12
    assert np.abs(F2[:, 24:27] - F[:, 24:27] @ Q.T).max() < 1e-12


def test_cutoff_counts_two_atoms():
    mol = G.single_gaussian_system("H2", 1.0, bond=3.0)
    F = guess.features(mol)
    # rows (0,0), (0,1), (1,1); H is element 0; f_c(3) = 1/2
    assert F[0, 33] == pytest.approx(0.5, abs=1e-15) and F[0, 34:37].sum() == 0
    assert F[1, 33] == pytest.approx(0.5, abs=1e-15) and F[1, 37] == pytest.approx(0.5, abs=1e-15)
    mol6 = G.single_gaussian_system("H2", 1.0, bond=6.0)
    assert guess.features(mol6)[0, 33] == 0.0
    # radial function k at R = mu_k is 1
    assert F[1, 8 + 0] == pytest.approx(math.exp(-((3.0 / (10 / 15)) ** 2)), rel=1e-14)


def test_block_round_trip():
    mol = G.batched_molecule(1003)
    rng = np.random.Generator(np.random.PCG64(6))
    A = rng.normal(size=(mol.n_bf, mol.n_bf))
    D = A + A.T
    T, M = guess.targets(mol, D)
    assert np.array_equal(guess.assemble(mol, T), D)
    first, count = guess.atom_functions(mol)
    assert M.sum() == sum(count[a] * count[b] for a, b in guess.pairs(mol))


def test_projection_properties():
    mol = G.batched_molecule(1003)
    S = core.one_electron(mol)[0]
    rng = np.random.Generator(np.random.PCG64(7))
    A = rng.normal(size=(mol.n_bf, mol.n_bf)) * 0.1
    Dp = guess.project(mol, A + A.T, S)
    assert np.abs(Dp @ S @ Dp - 2.0 * Dp).max() < 1e-9 * np.abs(Dp).max()
    assert abs(np.sum(Dp * S) - mol.n_electrons) < 1e-9
    # an idempotent density with the right electron count is a fixed point
    D0 = scf.RHF(mol).core_guess()
    assert np.abs(guess.project(mol, D0, S) - D0).max() < 1e-9


def test_commutator_residual_vanishes_at_convergence():
    mol = G.random_small_molecule(1)
    r = scf.RHF(mol, conv_tol=1e-11, max_iter=200).run()
    assert r["converged"]
    assert guess.commutator_residual(mol, r["D"]) < 1e-4
    assert guess.commutator_residual(mol, scf.RHF(mol).core_guess()) > 1e-2
