"""Brute-force numerical integrals used to pin the oracle.

Independent of the oracle's McMurchie-Davidson route: every integral here is
the defining integral evaluated numerically.  Polynomial-times-Gaussian
integrands are integrated exactly by Gauss-Hermite quadrature after the
quadratic form in the exponent is whitened; the Coulomb kernel is written as
1/r = (2/sqrt(pi)) int_0^inf exp(-t^2 r^2) dt and the t integral is done by
adaptive quadrature (scipy).
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate

_GH_X, _GH_W = np.polynomial.hermite.hermgauss(24)


def cart_components(l):
    out = []
    for lx in range(l, -1, -1):
        for ly in range(l - lx, -1, -1):
            out.append((lx, ly, l - lx - ly))
    return out


def basis_functions(mol, coefs):
    """List of (centre, (lx,ly,lz), exps, full coefficients) per function.

    ``coefs`` is the [nprim, 6] array of normalised coefficients to test."""
    funcs = []
    p0 = 0
    for s in range(mol.n_shells):
        l = int(mol.shell_l[s])
        k = int(mol.shell_nprim[s])
        A = mol.xyz[mol.shell_atom[s]]
        for c, lmn in enumerate(cart_components(l)):
            funcs.append((A, lmn, mol.exps[p0:p0 + k], coefs[p0:p0 + k, c]))
        p0 += k
    return funcs


def _gauss_1d(poly, terms):
    """int poly(x) exp(-sum_k e_k (x - X_k)^2) dx for terms [(e_k, X_k)].

    The exponent is rewritten as E (x - m)^2 + sum_k e_k (X_k - m)^2 (no
    cancellation), then Gauss-Hermite is exact for polynomial degree < 48."""
    a = sum(e for e, _ in terms)
    m = sum(e * X for e, X in terms) / a
    rest = sum(e * (X - m) ** 2 for e, X in terms)
    x = m + _GH_X / math.sqrt(a)
    return float(np.sum(_GH_W * poly(x))) / math.sqrt(a) * math.exp(-rest)


def _t_integral(f):
    """int_0^inf f(t) dt via t = s/(1-s); f decays like t^-3 so the s integrand
    is smooth on [0, 1]."""
    g = lambda s: 0.0 if s >= 1.0 else f(s / (1.0 - s)) / (1.0 - s) ** 2  # noqa: E731
    with warnings.catch_warnings():
        # quad's own error estimate is pessimistic near 1e-12; the tests'
        # tolerances decide, not the estimate
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        v, _ = integrate.quad(g, 0.0, 1.0, epsabs=0.0, epsrel=1e-12, limit=400)
    return v


def overlap_1d(i, A, a, j, B, b):
    return _gauss_1d(lambda x: (x - A) ** i * (x - B) ** j, [(a, A), (b, B)])


def kinetic_1d(i, A, a, j, B, b):
    """int g_i(x) d^2/dx^2 g_j(x) dx (the second derivative written out)."""
    def d2(x):
        y = x - B
        val = -2.0 * b * (2 * j + 1) * y ** j + 4.0 * b * b * y ** (j + 2)
        if j >= 2:
            val = val + j * (j - 1) * y ** (j - 2)
        return (x - A) ** i * val
    return _gauss_1d(d2, [(a, A), (b, B)])


def overlap(f, g):
    (A, la, ea, ca), (B, lb, eb, cb) = f, g
    tot = 0.0
    for a, da in zip(ea, ca):
        for b, db in zip(eb, cb):
            tot += da * db * np.prod([overlap_1d(la[x], A[x], a, lb[x], B[x], b) for x in range(3)])
    return tot


def kinetic(f, g):
    (A, la, ea, ca), (B, lb, eb, cb) = f, g
    tot = 0.0
    for a, da in zip(ea, ca):
        for b, db in zip(eb, cb):
            s = [overlap_1d(la[x], A[x], a, lb[x], B[x], b) for x in range(3)]
            k = [kinetic_1d(la[x], A[x], a, lb[x], B[x], b) for x in range(3)]
            tot += da * db * -0.5 * (k[0] * s[1] * s[2] + s[0] * k[1] * s[2] + s[0] * s[1] * k[2])
    return tot


def nuclear(f, g, C, Z):
    """-Z int f g / |r - C| by the Gauss transform of 1/r."""
    (A, la, ea, ca), (B, lb, eb, cb) = f, g
    tot = 0.0
    for a, da in zip(ea, ca):
        for b, db in zip(eb, cb):
            def integrand(t):
                t2 = t * t
                val = 1.0
                for x in range(3):
                    val *= _gauss_1d(lambda y: (y - A[x]) ** la[x] * (y - B[x]) ** lb[x],
                                     [(a, A[x]), (b, B[x]), (t2, C[x])])
                return val
            v = _t_integral(integrand)
            tot += da * db * (2.0 / math.sqrt(math.pi)) * v
    return -Z * tot


def _pair_2d(i, A, a, j, B, b, k, C, c, l, D, d, t2):
    """int int (x1-A)^i (x1-B)^j (x2-C)^k (x2-D)^l
       exp(-a(x1-A)^2 - b(x1-B)^2 - t2 (x1-x2)^2 - c(x2-C)^2 - d(x2-D)^2)."""
    M = np.array([[a + b + t2, -t2], [-t2, c + d + t2]])
    h = np.array([a * A + b * B, c * C + d * D])
    m = np.linalg.solve(M, h)
    const = a * A * A + b * B * B + c * C * C + d * D * D - h @ m
    Lc = np.linalg.cholesky(M)          # M = L L^T
    Linv_T = np.linalg.inv(Lc).T
    gx, gw = np.polynomial.hermite.hermgauss(12)
    w1, w2 = np.meshgrid(gx, gx, indexing="ij")
    ww = np.outer(gw, gw)
    z = m[:, None, None] + np.einsum("ij,jab->iab", Linv_T, np.stack([w1, w2]))
    x1, x2 = z[0], z[1]
    f = (x1 - A) ** i * (x1 - B) ** j * (x2 - C) ** k * (x2 - D) ** l
    return float(np.sum(ww * f)) / (Lc[0, 0] * Lc[1, 1]) * math.exp(-const)


def eri(f1, f2, f3, f4):
    """(f1 f2 | f3 f4) by the Gauss transform of 1/r12 (primitive sums)."""
    tot = 0.0
    for a, da in zip(f1[2], f1[3]):
        for b, db in zip(f2[2], f2[3]):
            for c, dc in zip(f3[2], f3[3]):
                for d, dd in zip(f4[2], f4[3]):
                    def integrand(t):
                        t2 = t * t
                        val = 1.0
                        for x in range(3):
                            val *= _pair_2d(f1[1][x], f1[0][x], a, f2[1][x], f2[0][x], b,
                                            f3[1][x], f3[0][x], c, f4[1][x], f4[0][x], d, t2)
                        return val
                    v = _t_integral(integrand)
                    tot += da * db * dc * dd * (2.0 / math.sqrt(math.pi)) * v
    return tot
