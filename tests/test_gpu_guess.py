"""GPU parity of the learned initial guess against the oracle: features,
density blocks and assembly (exact), the BF16 perceptron forward and
gradient (the oracle emulating the same BF16 rounding points), one Adam
step, the natural-orbital projection and the residual judge; plus a
property check that training lowers the loss."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import announce, dev, host, need_gpu, zeros  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import guess as og  # noqa: E402
from oracle import scf as oscf  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEEDS = (1013, 1023, 1007)


def f32dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32), device="cuda")


@pytest.fixture(scope="module")
def setup():
    mess = need_gpu()
    mols = [G.batched_molecule(s) for s in SEEDS] + [G.random_small_molecule(1)]
    announce(f"learned guess batch nbf {[m.n_bf for m in mols]}")
    B = mess.mess_batch_create(mols)
    return mess, mols, B


def _oracle_rows(mols, fn):
    return np.concatenate([fn(m) for m in mols])


def test_features(setup):
    mess, mols, B = setup
    n = mess.mess_guess_rows(B)
    ref = _oracle_rows(mols, og.features)
    assert n == ref.shape[0]
    X = torch.zeros(n, 64, dtype=torch.float32, device="cuda")
    mess.mess_guess_features(B, X)
    got = X.cpu().numpy()
    # FP64 features rounded to FP32 on both sides; a one-ulp difference of
    # exp or cos before rounding may remain
    assert np.all(np.abs(got - ref.astype(np.float32)) <= 2.4e-7 * np.maximum(1.0, np.abs(ref)))


def test_targets_and_assembly(setup):
    mess, mols, B = setup
    rng = np.random.Generator(np.random.PCG64(3))
    Ds = []
    for m in mols:
        A = rng.normal(size=(m.n_bf, m.n_bf))
        Ds.append(A + A.T)
    Dp = dev(np.concatenate([d.ravel() for d in Ds]))
    n = mess.mess_guess_rows(B)
    T = torch.zeros(n, 128, dtype=torch.float32, device="cuda")
    M = torch.zeros_like(T)
    mess.mess_guess_targets(B, Dp, T, M)
    Tr = np.concatenate([og.targets(m, d)[0] for m, d in zip(mols, Ds)])
    Mr = np.concatenate([og.targets(m, d)[1] for m, d in zip(mols, Ds)])
    assert np.array_equal(T.cpu().numpy(), Tr.astype(np.float32))
    assert np.array_equal(M.cpu().numpy(), Mr.astype(np.float32))
    # assembly of arbitrary outputs
    Y = rng.normal(size=(n, 128)).astype(np.float32)
    D = zeros(B.packed)
    mess.mess_guess_assemble(B, f32dev(Y), D)
    got = host(D)
    r0 = 0
    for k, m in enumerate(mols):
        nr = len(og.pairs(m))
        want = og.assemble(m, Y[r0:r0 + nr].astype(np.float64))
        blk = got[B.mol_moff[k]:B.mol_moff[k + 1]].reshape(m.n_bf, m.n_bf)
        assert np.array_equal(blk, want), k
        r0 += nr


def _data(n=300, seed=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.normal(size=(n, 64)).astype(np.float32)
    T = (rng.normal(size=(n, 128)) * 0.1).astype(np.float32)
    M = (rng.uniform(size=(n, 128)) < 0.6).astype(np.float32)
    p = G.mlp_initial_params(1)
    p[og.SHAPES[0][0] * og.SHAPES[0][1]:][:256] = rng.normal(size=256) * 0.1  # non-zero b1
    return p, X, T, M


def test_forward_matches_bf16_oracle():
    mess = need_gpu()
    p, X, T, M = _data()
    mlp = mess.Mlp(p)
    Y = torch.zeros(X.shape[0], 128, dtype=torch.float32, device="cuda")
    mlp.forward(f32dev(X), Y)
    got = Y.cpu().numpy().astype(np.float64)
    ref, _ = og.forward_bf16(p.astype(np.float64), X.astype(np.float64))
    err = np.abs(got - ref)
    scale = np.abs(ref).max()
    announce(f"forward: max err {err.max():.3e} (max |Y| {scale:.3e}), median {np.median(err):.3e}, "
             f"frac>1e-5 rel {np.mean(err > 1e-5 * scale):.4f}")
    # FP32 sums in a different order, and the rare BF16 rounding of a hidden
    # activation that falls the other side of a rounding boundary (2^-8
    # relative each): bounded by a few such flips feeding each output
    assert np.median(err) <= 1e-6 * scale
    assert err.max() <= 2e-3 * scale


def test_gradient_matches_bf16_oracle():
    mess = need_gpu()
    p, X, T, M = _data()
    mlp = mess.Mlp(p)
    g = torch.zeros(mess.MESS_MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = mlp.grad(f32dev(X), f32dev(T), f32dev(M), g)
    Lr, gr = og.loss_and_grad_bf16(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                                   M.astype(np.float64))
    gg = g.cpu().numpy().astype(np.float64)
    assert abs(loss - Lr) <= 1e-5 * Lr
    offs = np.cumsum([0] + [int(np.prod(s)) for s in og.SHAPES])
    for t in range(6):
        a, b = offs[t], offs[t + 1]
        e = np.abs(gg[a:b] - gr[a:b])
        sc = np.abs(gr[a:b]).max()
        announce(f"grad tensor {t}: max err {e.max():.3e} (max |g| {sc:.3e}) median {np.median(e):.3e}")
        assert np.median(e) <= 1e-4 * sc, t
        assert e.max() <= 2e-3 * sc, t
    # the gradient points downhill for the exact loss as well
    L0, gexact = og.loss_and_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                                  M.astype(np.float64))
    assert np.dot(gg, gexact) > 0.9 * np.linalg.norm(gg) * np.linalg.norm(gexact)


def test_adam_step_and_training_lowers_loss():
    mess = need_gpu()
    p, X, T, M = _data()
    mlp = mess.Mlp(p)
    Xd, Td, Md = f32dev(X), f32dev(T), f32dev(M)
    l0 = mlp.train_step(Xd, Td, Md, lr=1e-3)
    p1 = mlp.params().astype(np.float64)
    Lr, gr = og.loss_and_grad_bf16(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                                   M.astype(np.float64))
    pr, _, _ = og.adam(p.astype(np.float64), np.zeros_like(gr), np.zeros_like(gr), gr, 1)
    # first Adam step moves each parameter by lr g/(|g| + eps): identical
    # wherever the gradient's sign is not in doubt
    sure = np.abs(gr) > 1e-2 * np.abs(gr).max()
    assert np.abs((p1 - p)[sure] - (pr - p)[sure]).max() <= 1e-6
    assert np.abs(p1 - pr).max() <= 2.0001e-3
    losses = [l0]
    for _ in range(60):
        losses.append(mlp.train_step(Xd, Td, Md, lr=1e-3))
    announce(f"training loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert losses[-1] < 0.5 * losses[0]


def test_projection(setup):
    mess, mols, B = setup
    rng = np.random.Generator(np.random.PCG64(9))
    Ds = []
    for m in mols:
        A = rng.normal(size=(m.n_bf, m.n_bf)) * 0.1
        Ds.append(A + A.T)
    D = dev(np.concatenate([d.ravel() for d in Ds]))
    mess.mess_guess_project(B, D)
    got = host(D)
    for k, m in enumerate(mols):
        want = og.project(m, Ds[k])
        blk = got[B.mol_moff[k]:B.mol_moff[k + 1]].reshape(m.n_bf, m.n_bf)
        assert np.abs(blk - want).max() <= 1e-9 * max(1.0, np.abs(want).max()), k


def test_judge(setup):
    mess, mols, B = setup
    rng = np.random.Generator(np.random.PCG64(10))
    cand, core_d = [], []
    for k, m in enumerate(mols):
        core_d.append(oscf.RHF(m).core_guess())
        if k % 2 == 0:
            A = rng.normal(size=(m.n_bf, m.n_bf)) * 0.1
            cand.append(og.project(m, A + A.T))          # a poor guess
        else:
            r = oscf.RHF(m, conv_tol=1e-9, max_iter=200).run()
            cand.append(r["D"])                           # the converged density
    D0 = dev(np.concatenate([d.ravel() for d in cand]))
    used = mess.mess_guess_judge(B, D0, schwarz_tol=0.0)
    got = host(D0)
    for k, m in enumerate(mols):
        want_keep = og.commutator_residual(m, cand[k]) < og.commutator_residual(m, core_d[k])
        assert bool(used[k]) == want_keep, k
        blk = got[B.mol_moff[k]:B.mol_moff[k + 1]].reshape(m.n_bf, m.n_bf)
        want = cand[k] if want_keep else core_d[k]
        assert np.abs(blk - want).max() <= 1e-9 * max(1.0, np.abs(want).max()), k
