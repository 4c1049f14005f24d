"""Learned initial density guess (oracle; FP64 NumPy; test infrastructure only).

The paper builds its Hartree-Fock and DFT energies as differentiable
functions so that learned components can be trained (sections 1 and 5); the
learned initial guess here is one such component, with every detail a
reading (restated in the design notes):

* One row per atom pair (A, B), A <= B, of one molecule, A-major order.
  Features, 42 used of 64: one-hot element of A and of B over (H, C, N, O);
  16 Gaussian radial functions exp(-((R_AB - mu_k)/sigma)^2), mu_k = k 10/15,
  sigma = 10/15 bohr; the unit vector u = (B - A)/R_AB (zero for A = B) and
  the six products u_x u_x, u_x u_y, u_x u_z, u_y u_y, u_y u_z, u_z u_z;
  per-element neighbour counts of A and of B, sum over other atoms C of
  f_c(R) = (cos(pi R / 6) + 1)/2 for R < 6 bohr; a self-pair flag.
* Perceptron 64 -> 256 -> 256 -> 128, SiLU z / (1 + e^-z) on the hidden
  layers; output k = 11 i + j is the density element between function i of
  A and function j of B (at most 11 functions per atom), masked to the
  block's real size.  Loss: mean squared error over the masked elements.
* Assembly: D[A_i, B_j] = D[B_j, A_i] = y_{11 i + j}; diagonal blocks take
  (y_{11 i + j} + y_{11 j + i}) / 2.
* Projection onto an idempotent density with the right electron count:
  D' = 2 S^-1/2 V V^T S^-1/2, V the n_occ eigenvectors of S^1/2 D S^1/2 of
  largest eigenvalue.
* Judge: keep D' only if its first commutator residual max|X^T(FDS - SDF)X|
  is below the core-Hamiltonian guess's; otherwise use the core guess.
* Arithmetic of the device kernels, emulated by the *_bf16 functions: every
  GEMM operand (inputs, weights, activations, back-propagated gradients) is
  rounded to BF16 (round to nearest even), products accumulate in FP32,
  biases, pre-activations and gradients are FP32; Adam (beta 0.9 / 0.999,
  eps 1e-8) updates FP32 master weights.
"""
from __future__ import annotations

import math

import numpy as np

from . import core

ELEMENTS = (1, 6, 7, 8)
N_IN, N_H, N_OUT, BLK = 64, 256, 128, 11
SHAPES = ((256, 64), (256,), (256, 256), (256,), (128, 256), (128,))
NPARAM = sum(int(np.prod(s)) for s in SHAPES)
RBF_MU = np.arange(16) * (10.0 / 15.0)
RBF_SIGMA = 10.0 / 15.0
R_CUT = 6.0


def _ncart(l):
    return (l + 1) * (l + 2) // 2


def atom_functions(mol):
    """(first function, count) per atom; atoms' functions must be contiguous."""
    nat = len(mol.Z)
    first = [-1] * nat
    count = [0] * nat
    bf = 0
    last = -1
    for s in range(len(mol.shell_l)):
        a = int(mol.shell_atom[s])
        if first[a] < 0:
            if a < last:
                raise ValueError("shells of an atom are not contiguous")
            first[a] = bf
        elif a != last:
            raise ValueError("shells of an atom are not contiguous")
        last = a
        n = _ncart(int(mol.shell_l[s]))
        count[a] += n
        bf += n
    if max(count) > BLK:
        raise ValueError("more than 11 functions on one atom")
    return np.array(first), np.array(count)


def pairs(mol):
    nat = len(mol.Z)
    return [(a, b) for a in range(nat) for b in range(a, nat)]


def features(mol) -> np.ndarray:
    xyz = np.asarray(mol.xyz, np.float64).reshape(-1, 3)
    Z = [int(z) for z in mol.Z]
    el = [ELEMENTS.index(z) for z in Z]
    nat = len(Z)
    R = np.linalg.norm(xyz[:, None, :] - xyz[None, :, :], axis=2)
    fc = np.where(R < R_CUT, 0.5 * (np.cos(np.pi * R / R_CUT) + 1.0), 0.0)
    counts = np.zeros((nat, 4))
    for a in range(nat):
        for c in range(nat):
            if c != a:
                counts[a, el[c]] += fc[a, c]
    rows = []
    for a, b in pairs(mol):
        f = np.zeros(N_IN)
        f[el[a]] = 1.0
        f[4 + el[b]] = 1.0
        r = R[a, b]
        f[8:24] = np.exp(-(((r - RBF_MU) / RBF_SIGMA) ** 2))
        if a != b:
            u = (xyz[b] - xyz[a]) / r
            f[24:27] = u
            f[27:33] = [u[0] * u[0], u[0] * u[1], u[0] * u[2], u[1] * u[1], u[1] * u[2], u[2] * u[2]]
        f[33:37] = counts[a]
        f[37:41] = counts[b]
        f[41] = 1.0 if a == b else 0.0
        rows.append(f)
    return np.array(rows)


def targets(mol, D):
    """(T, M): the pair blocks of D and their masks, [n_pairs, 128]."""
    first, count = atom_functions(mol)
    P = pairs(mol)
    T = np.zeros((len(P), N_OUT))
    M = np.zeros((len(P), N_OUT))
    for r, (a, b) in enumerate(P):
        for i in range(count[a]):
            for j in range(count[b]):
                T[r, BLK * i + j] = D[first[a] + i, first[b] + j]
                M[r, BLK * i + j] = 1.0
    return T, M


def assemble(mol, Y):
    first, count = atom_functions(mol)
    N = mol.n_bf
    D = np.zeros((N, N))
    for r, (a, b) in enumerate(pairs(mol)):
        for i in range(count[a]):
            for j in range(count[b]):
                if a == b:
                    v = 0.5 * (Y[r, BLK * i + j] + Y[r, BLK * j + i])
                else:
                    v = Y[r, BLK * i + j]
                D[first[a] + i, first[b] + j] = v
                D[first[b] + j, first[a] + i] = v
    return D


def project(mol, D, S=None):
    """Idempotent density with n_occ = N_e/2 natural orbitals of D (metric S)."""
    if S is None:
        S = core.one_electron(mol)[0]
    s, U = np.linalg.eigh(S)
    Sh = (U * np.sqrt(s)) @ U.T
    Smh = (U / np.sqrt(s)) @ U.T
    w, V = np.linalg.eigh(Sh @ D @ Sh)
    nocc = mol.n_electrons // 2
    Vo = V[:, len(w) - nocc:]
    return 2.0 * Smh @ Vo @ Vo.T @ Smh


# ------------------------------------------------------------ perceptron

def unpack(params):
    out, k = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(params[k:k + n], np.float64).reshape(s))
        k += n
    return out


def pack(arrays):
    return np.concatenate([np.asarray(a, np.float64).ravel() for a in arrays])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def forward(params, X):
    """Exact FP64 forward: returns Y and the cache (Z1, H1, Z2, H2)."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    Z1 = X @ W1.T + b1
    H1 = silu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = silu(Z2)
    return H2 @ W3.T + b3, (X, Z1, H1, Z2, H2)


def loss_and_grad(params, X, T, M):
    """Masked MSE and its exact FP64 gradient (flat, parameter order)."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    Y, (X, Z1, H1, Z2, H2) = forward(params, X)
    nm = M.sum()
    L = float(np.sum(M * (Y - T) ** 2) / nm)
    dY = 2.0 * M * (Y - T) / nm
    dW3, db3 = dY.T @ H2, dY.sum(0)
    dZ2 = (dY @ W3) * dsilu(Z2)
    dW2, db2 = dZ2.T @ H1, dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * dsilu(Z1)
    dW1, db1 = dZ1.T @ X, dZ1.sum(0)
    return L, pack([dW1, db1, dW2, db2, dW3, db3])


def _mm(A, B):
    """FP32 result of a product of BF16 operands (exact sums, then rounded)."""
    return f32(bf16(A) @ bf16(B))


def forward_bf16(params, X):
    """The device forward: BF16 GEMM operands, FP32 accumulation and bias."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    Z1 = f32(_mm(X, W1.T) + f32(b1))
    H1 = f32(silu(Z1))
    Z2 = f32(_mm(H1, W2.T) + f32(b2))
    H2 = f32(silu(Z2))
    Y = f32(_mm(H2, W3.T) + f32(b3))
    return Y, (X, Z1, H1, Z2, H2)


def loss_and_grad_bf16(params, X, T, M):
    """The device backward (same rounding points as forward_bf16)."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    Y, (X, Z1, H1, Z2, H2) = forward_bf16(params, X)
    nm = M.sum()
    L = float(np.sum(M * (Y - T) ** 2) / nm)
    dY = f32(2.0 * M * (Y - T) / nm)
    dW3, db3 = _mm(dY.T, H2), f32(dY.sum(0))
    dZ2 = f32(_mm(dY, W3) * dsilu(Z2))
    dW2, db2 = _mm(dZ2.T, H1), f32(dZ2.sum(0))
    dZ1 = f32(_mm(dZ2, W2) * dsilu(Z1))
    dW1, db1 = _mm(dZ1.T, X), f32(dZ1.sum(0))
    return L, pack([dW1, db1, dW2, db2, dW3, db3])


def adam(params, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def commutator_residual(mol, D, S=None, H=None):
    """max |X^T (F D S - S D F) X| of the Hartree-Fock Fock matrix at D."""
    if S is None or H is None:
        S, T, V = core.one_electron(mol)
        H = T + V
    J, K = core.jk_from_dense(core.eri_dense(mol), D)
    F = H + J - 0.5 * K
    s, U = np.linalg.eigh(S)
    X = (U / np.sqrt(s)) @ U.T
    return float(np.abs(X.T @ (F @ D @ S - S @ D @ F) @ X).max())


def rbf_width():
    return RBF_SIGMA


def cutoff(r):
    return 0.5 * (math.cos(math.pi * r / R_CUT) + 1.0) if r < R_CUT else 0.0
