"""ctypes binding of the C oracle (``mess_oracle.c``) and plain-sum J/K.

Test infrastructure only; see the package docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mess_oracle.c")
# FP64 oracle, and the same source in x87 extended precision (long double,
# 64-bit mantissa) used only to arbitrate rounding-level disagreements.
_LIBS = {"fp64": (os.path.join(_HERE, "libmess_oracle.so"), []),
         "ext": (os.path.join(_HERE, "libmess_oracle_ext.so"), ["-DOR_REAL=long double"])}
_lib = {}
_ext = False


class extended_precision:
    """Context manager: oracle calls inside use the long-double build."""

    def __enter__(self):
        global _ext
        self._old, _ext = _ext, True

    def __exit__(self, *a):
        global _ext
        _ext = self._old


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP), FP64 and extended variants."""
    for path, defs in _LIBS.values():
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared"] + defs +
                                  ["-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIBS["fp64"][0]


def lib():
    key = "ext" if _ext else "fp64"
    if key not in _lib:
        build()
        L = ctypes.CDLL(_LIBS[key][0])
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        mol = [ctypes.c_int, i32p, f64p, ctypes.c_int, i32p, i32p, i32p, f64p, f64p]
        L.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, f64p]
        L.oracle_boys.restype = None
        L.oracle_nuclear_repulsion.argtypes = [ctypes.c_int, i32p, f64p]
        L.oracle_nuclear_repulsion.restype = ctypes.c_double
        L.oracle_coefficients.argtypes = mol + [f64p]
        L.oracle_one_electron.argtypes = mol + [f64p, f64p, f64p]
        L.oracle_eri_shell_quartet.argtypes = mol + [ctypes.c_int] * 4 + [f64p]
        L.oracle_eri_quartet_list.argtypes = mol + [ctypes.c_long, i32p, i64p, f64p]
        L.oracle_eri_dense.argtypes = mol + [f64p]
        L.oracle_schwarz.argtypes = mol + [f64p]
        L.oracle_jk_unique.argtypes = mol + [f64p, ctypes.c_double, f64p, f64p,
                                             ctypes.POINTER(ctypes.c_longlong)]
        L.oracle_jk_elements.argtypes = mol + [f64p, ctypes.c_int, i32p, i32p, f64p, f64p]
        _lib[key] = L
    return _lib[key]


def _mol_args(m):
    return (int(m.n_atoms), np.ascontiguousarray(m.Z, np.int32),
            np.ascontiguousarray(m.xyz, np.float64).reshape(-1), int(m.n_shells),
            np.ascontiguousarray(m.shell_atom, np.int32), np.ascontiguousarray(m.shell_l, np.int32),
            np.ascontiguousarray(m.shell_nprim, np.int32), np.ascontiguousarray(m.exps, np.float64),
            np.ascontiguousarray(m.coefs, np.float64))


def _check(rc):
    if rc != 0:
        raise ValueError("oracle rejected the basis (l outside 0..2 or bad primitive count)")


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def boys(nmax: int, T: float) -> np.ndarray:
    """F_0..F_nmax at T."""
    out = np.zeros(nmax + 1)
    lib().oracle_boys(int(nmax), float(T), out)
    return out


def nuclear_repulsion(m) -> float:
    """E_nuc = sum_{A<B} Z_A Z_B / R_AB (the term added to the electronic energy)."""
    return float(lib().oracle_nuclear_repulsion(int(m.n_atoms), np.ascontiguousarray(m.Z, np.int32),
                                                np.ascontiguousarray(m.xyz, np.float64).reshape(-1)))


def coefficients(m) -> np.ndarray:
    """Normalised primitive coefficients, shape [sum nprim, 6] (per Cartesian component)."""
    out = np.zeros((int(m.shell_nprim.sum()), 6))
    _check(lib().oracle_coefficients(*_mol_args(m), out.reshape(-1)))
    return out


def one_electron(m):
    """Overlap S (eq. 3), kinetic T and nuclear attraction V, each N x N."""
    N = m.n_bf
    S, T, V = (np.zeros((N, N)) for _ in range(3))
    _check(lib().oracle_one_electron(*_mol_args(m), S.reshape(-1), T.reshape(-1), V.reshape(-1)))
    return S, T, V


def eri_shell_quartet(m, a, b, c, d) -> np.ndarray:
    l = m.shell_l
    out = np.zeros((ncart(l[a]), ncart(l[b]), ncart(l[c]), ncart(l[d])))
    _check(lib().oracle_eri_shell_quartet(*_mol_args(m), int(a), int(b), int(c), int(d), out.reshape(-1)))
    return out


def eri_quartet_list(m, quartets) -> list:
    """Blocks for an int array of shell quartets [nq, 4]."""
    q = np.ascontiguousarray(quartets, dtype=np.int32).reshape(-1, 4)
    l = m.shell_l
    sizes = np.array([ncart(l[a]) * ncart(l[b]) * ncart(l[c]) * ncart(l[d]) for a, b, c, d in q],
                     dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    out = np.zeros(int(sizes.sum()) if len(sizes) else 1)
    _check(lib().oracle_eri_quartet_list(*_mol_args(m), int(len(q)), q.reshape(-1), offs, out))
    blocks = []
    for (a, b, c, d), o, s in zip(q, offs, sizes):
        blocks.append(out[o:o + s].reshape(ncart(l[a]), ncart(l[b]), ncart(l[c]), ncart(l[d])))
    return blocks


def eri_dense(m) -> np.ndarray:
    """Full (ij|kl) tensor, every shell quartet computed independently."""
    N = m.n_bf
    out = np.zeros((N, N, N, N))
    _check(lib().oracle_eri_dense(*_mol_args(m), out.reshape(-1)))
    return out


def schwarz(m) -> np.ndarray:
    """Q[a, b] = sqrt(max over the block of |(ab|ab)|), shell-level."""
    out = np.zeros((m.n_shells, m.n_shells))
    _check(lib().oracle_schwarz(*_mol_args(m), out.reshape(-1)))
    return out


def jk_from_dense(eri: np.ndarray, D: np.ndarray):
    """J_ij = sum_kl (ij|kl) D_kl and K_ij = sum_kl (ik|jl) D_kl: the definitions."""
    J = np.einsum("ijkl,kl->ij", eri, D)
    K = np.einsum("ikjl,kl->ij", eri, D)
    return J, K


def jk_unique(m, D: np.ndarray, tau: float = 0.0):
    """J, K from unique shell quartets with the 8-permutation update rule.

    Returns (J, K, number of shell quartets evaluated)."""
    N = m.n_bf
    J, K = np.zeros((N, N)), np.zeros((N, N))
    cnt = ctypes.c_longlong(0)
    _check(lib().oracle_jk_unique(*_mol_args(m), np.ascontiguousarray(D, np.float64).reshape(-1),
                                  float(tau), J.reshape(-1), K.reshape(-1), ctypes.byref(cnt)))
    return J, K, int(cnt.value)


def jk_elements(m, D: np.ndarray, mu, nu):
    """Selected J[mu, nu], K[mu, nu] computed from their defining sums."""
    mu = np.ascontiguousarray(mu, dtype=np.int32)
    nu = np.ascontiguousarray(nu, dtype=np.int32)
    Jo, Ko = np.zeros(len(mu)), np.zeros(len(mu))
    _check(lib().oracle_jk_elements(*_mol_args(m), np.ascontiguousarray(D, np.float64).reshape(-1),
                                    int(len(mu)), mu, nu, Jo, Ko))
    return Jo, Ko
