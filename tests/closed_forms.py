"""Textbook closed forms used as pins (no oracle code involved).

* (ss|ss) of normalised s primitives: Gaussian product theorem and F_0.
* Restricted Hartree-Fock energy of H2 in a minimal basis of one
  normalised s Gaussian (exponent alpha) per atom, bond length R: by
  symmetry the occupied orbital is (phi_1 + phi_2) / sqrt(2 (1 + S)), so
  E = 2 (h11 + h12) / (1 + S)
      + [(11|11) + (11|22) + 2 (12|12) + 4 (11|12)] / (2 (1 + S)^2) + 1/R
  (Szabo-Ostlund minimal-basis H2 algebra).
"""
import math

import numpy as np


def f0(T):
    return 1.0 if T == 0 else 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))


def ss_eri(a, A, b, B, c, C, d, D):
    """(ss|ss) of normalised s primitives."""
    A, B, C, D = map(np.asarray, (A, B, C, D))
    p, q = a + b, c + d
    P, Qc = (a * A + b * B) / p, (c * C + d * D) / q
    Kab = math.exp(-a * b / p * np.sum((A - B) ** 2))
    Kcd = math.exp(-c * d / q * np.sum((C - D) ** 2))
    rho = p * q / (p + q)
    T = rho * np.sum((P - Qc) ** 2)
    norm = np.prod([(2 * x / math.pi) ** 0.75 for x in (a, b, c, d)])
    return 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * Kab * Kcd * f0(T) * norm


def h2_minimal_energy(alpha, R):
    A, B = np.zeros(3), np.array([0.0, 0.0, R])
    S12 = math.exp(-alpha * R * R / 2)
    mu = alpha / 2
    T11, T12 = 1.5 * alpha, mu * (3 - 2 * mu * R * R) * S12
    c = 2 * math.sqrt(2 * alpha / math.pi)
    V11 = -c * (1 + f0(2 * alpha * R * R))
    V12 = -c * S12 * 2 * f0(2 * alpha * (R / 2) ** 2)
    h11, h12 = T11 + V11, T12 + V12
    g = lambda P, Qq, Rr, Ss: ss_eri(alpha, P, alpha, Qq, alpha, Rr, alpha, Ss)  # noqa: E731
    J = (g(A, A, A, A) + g(A, A, B, B) + 2 * g(A, B, A, B) + 4 * g(A, A, A, B)) / (2 * (1 + S12) ** 2)
    return 2 * (h11 + h12) / (1 + S12) + J + 1.0 / R
