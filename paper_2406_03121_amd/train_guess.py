"""Train the learned initial-guess perceptron on one GPU.

1. Converged densities of seeded molecules (3..20 atoms of H, C, N, O, one
   fixed per-element basis) from the batched SCF (FP64, Schwarz 1e-10).
2. Pair features and density blocks of every converged molecule
   (mess_guess_features / mess_guess_targets), kept in device memory.
3. Mini-batch Adam on the masked block loss with the BF16 matrix-core
   forward/backward (mess_mlp_train_step).
4. Evaluation on the test molecules: predicted blocks -> assembled density
   -> natural-orbital projection -> residual judge against the core guess
   -> batched SCF, against the same SCF from the core guess alone.

Usage: python -m paper_2406_03121_amd.train_guess [--train N] [--epochs E]
       [--out FILE.npz]
Writes the FP32 parameters (numpy .npz, key "params") and prints one JSON
line of training and evaluation figures.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(msg):
    print(f"[train_guess] {msg}", file=sys.stderr, flush=True)


def converged_blocks(mess, torch, mols, tau, conv, max_steps):
    """Features, targets and masks (device tensors) of the molecules whose
    batched SCF converged, and the count of those."""
    B = mess.mess_batch_create(mols)
    st = mess.mess_batch_scf_create(B, schwarz_tol=tau, conv_tol=conv, diis_size=8, use_graph=True)
    for k in range(max_steps):
        mess.mess_batch_scf_step(st)
        if k % 5 == 4 or k == max_steps - 1:
            s = mess.mess_batch_scf_status(st)
            if s["n_converged"] == len(mols):
                break
    s = mess.mess_batch_scf_status(st)
    D = torch.zeros(B.packed, dtype=torch.float64, device="cuda")
    mess.mess_batch_scf_density(st, D)
    st.close()
    n = mess.mess_guess_rows(B)
    X = torch.zeros(n, 64, dtype=torch.float32, device="cuda")
    T = torch.zeros(n, 128, dtype=torch.float32, device="cuda")
    M = torch.zeros_like(T)
    mess.mess_guess_features(B, X)
    mess.mess_guess_targets(B, D, T, M)
    # rows of molecules that converged
    nat = np.array([len(m.Z) for m in mols])
    rows_per = nat * (nat + 1) // 2
    keep = np.repeat(s["converged"], rows_per)
    idx = torch.as_tensor(np.nonzero(keep)[0], device="cuda")
    return X[idx], T[idx], M[idx], int(s["converged"].sum())


def predict_density(mess, torch, mlp, B):
    n = mess.mess_guess_rows(B)
    X = torch.zeros(n, 64, dtype=torch.float32, device="cuda")
    Y = torch.zeros(n, 128, dtype=torch.float32, device="cuda")
    mess.mess_guess_features(B, X)
    mlp.forward(X, Y)
    D = torch.zeros(B.packed, dtype=torch.float64, device="cuda")
    mess.mess_guess_assemble(B, Y, D)
    mess.mess_guess_project(B, D)
    return D


def scf_convergence(mess, torch, B, D0, tau, conv, steps):
    """Per-step converged counts and each molecule's converging step (-1: not)."""
    st = mess.mess_batch_scf_create(B, schwarz_tol=tau, conv_tol=conv, diis_size=8, D0=D0, use_graph=True)
    at = np.full(B.n_mol, -1)
    counts = []
    t0 = time.perf_counter()
    for k in range(steps):
        mess.mess_batch_scf_step(st)
        s = mess.mess_batch_scf_status(st)
        newly = s["converged"] & (at < 0)
        at[newly] = k + 1
        counts.append(int(s["n_converged"]))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    e = s["energy"]
    st.close()
    return counts, at, el, e


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=10000)
    ap.add_argument("--val", type=int, default=500)
    ap.add_argument("--test", type=int, default=1024)
    ap.add_argument("--chunk", type=int, default=2048)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tau", type=float, default=1e-10)
    ap.add_argument("--conv-data", type=float, default=1e-7)
    ap.add_argument("--data-steps", type=int, default=20)
    ap.add_argument("--eval-steps", type=int, default=30)
    ap.add_argument("--out", default="guess_mlp.npz")
    ap.add_argument("--init", default=None, help=".npz with parameters to start from")
    a = ap.parse_args(argv)

    import torch
    from mess_inputs import generators as G
    from paper_2406_03121_amd import mess
    torch.cuda.init()
    tr_seeds, va_seeds, te_seeds = G.guess_train_seeds()
    tr_seeds = list(tr_seeds)[:a.train]
    va_seeds = list(va_seeds)[:a.val]
    te_seeds = list(te_seeds)[:a.test]

    t0 = time.perf_counter()
    parts, nconv = [], 0
    for c0 in range(0, len(tr_seeds), a.chunk):
        mols = [G.batched_molecule(s) for s in tr_seeds[c0:c0 + a.chunk]]
        X, T, M, nc = converged_blocks(mess, torch, mols, a.tau, a.conv_data, a.data_steps)
        parts.append((X, T, M))
        nconv += nc
        log(f"training data: molecules {c0 + len(mols)}/{len(tr_seeds)}, converged {nconv}, "
            f"{time.perf_counter() - t0:.0f} s")
    X = torch.cat([p[0] for p in parts])
    T = torch.cat([p[1] for p in parts])
    M = torch.cat([p[2] for p in parts])
    del parts
    vmols = [G.batched_molecule(s) for s in va_seeds]
    Xv, Tv, Mv, nv = converged_blocks(mess, torch, vmols, a.tau, a.conv_data, a.data_steps)
    data_s = time.perf_counter() - t0
    log(f"rows: train {X.shape[0]}, validation {Xv.shape[0]} ({data_s:.0f} s)")

    p0 = np.load(a.init)["params"] if a.init else G.mlp_initial_params(0)
    mlp = mess.Mlp(p0)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    n = X.shape[0]
    history = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    steps = 0
    for ep in range(a.epochs):
        perm = torch.randperm(n, device="cuda", generator=gen)
        for b0 in range(0, n - a.batch + 1, a.batch):
            idx = perm[b0:b0 + a.batch]
            mlp.train_step(X[idx].contiguous(), T[idx].contiguous(), M[idx].contiguous(), lr=a.lr,
                           want_loss=False)
            steps += 1
        lt = mlp.grad(X[:200000].contiguous(), T[:200000].contiguous(), M[:200000].contiguous())
        lv = mlp.grad(Xv, Tv, Mv)
        history.append((ep + 1, lt, lv))
        log(f"epoch {ep + 1}: train loss {lt:.4e}  validation loss {lv:.4e}")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    params = mlp.params()
    np.savez(a.out, params=params)
    log(f"wrote {a.out}")

    # evaluation on the test molecules
    tmols = [G.batched_molecule(s) for s in te_seeds]
    Bt = mess.mess_batch_create(tmols)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    D = predict_density(mess, torch, mlp, Bt)
    used = mess.mess_guess_judge(Bt, D, schwarz_tol=a.tau)
    torch.cuda.synchronize()
    guess_s = time.perf_counter() - t2
    c_learn, at_learn, el_learn, e_learn = scf_convergence(mess, torch, Bt, D, a.tau, 1e-8, a.eval_steps)
    c_core, at_core, el_core, e_core = scf_convergence(mess, torch, Bt, None, a.tau, 1e-8, a.eval_steps)
    both = (at_learn > 0) & (at_core > 0)
    same = both & (np.abs(e_learn - e_core) < 1e-6)
    out = {
        "train_molecules": len(tr_seeds), "train_converged": nconv, "train_rows": int(n),
        "validation_rows": int(Xv.shape[0]), "data_seconds": data_s,
        "epochs": a.epochs, "adam_steps": steps, "train_seconds": train_s,
        "train_rows_per_s": steps * a.batch / train_s,
        "train_tflops_bf16": steps * a.batch * 6 * 114688 / train_s / 1e12,
        "loss_history": history,
        "test_molecules": len(tmols), "learned_kept": int(used.sum()), "fallback_rate": float(1 - used.mean()),
        "guess_seconds": guess_s,
        "converged_per_step_learned": c_learn, "converged_per_step_core": c_core,
        "mean_steps_learned": float(at_learn[both].mean()) if both.any() else None,
        "mean_steps_core": float(at_core[both].mean()) if both.any() else None,
        "same_energy_fraction": float(same.sum() / max(1, both.sum())),
        "scf_seconds_learned": el_learn, "scf_seconds_core": el_core,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
