"""Seeded synthetic workloads: atoms, positions and contracted Cartesian shells.

Every array returned here is an *input*: positions in bohr, element numbers,
shell layout (atom, angular momentum l, primitive count) and the raw
primitive exponents / contraction coefficients.  Normalisation and every
integral are the job of the consumers (the oracle and the HIP library).

Workload recipes (all drawn from ``numpy.random.Generator(PCG64(seed))``):

* ``hco6_sp``: 6 atoms from {H, C, O} uniform in a 6-bohr cube, minimum
  separation 1.8 bohr, every atom carries shells {s, s, p} with 3 primitives
  each, exponents log-uniform in [0.1, 50], coefficients uniform in (0, 1]
  -> 30 basis functions.  Elements are redrawn until the electron count is even.
* ``water60_spd``: 20 water molecules (O-H 1.81 bohr, H-O-H 104.5 deg) at
  uniformly random orientations, O centres uniform in an 18-bohr cube with
  O-O >= 5 bohr and every intermolecular atom pair >= 1.8 bohr.  O carries
  {s, s, p, d}, H carries {s, s}; 3..6 primitives per shell, exponents
  log-uniform in [0.05, 5000], coefficients uniform in (0, 1] -> 300 functions.
* ``mol3to20_spd``: 3..20 atoms from {H, C, N, O} in a cube of side
  6 * (n/6)^(1/3) bohr, min separation 1.8 bohr, one fixed per-element basis
  (H {s,s}, C/N {s,s,p}, O {s,s,p,d}, drawn once from seed 7 with the
  water60 exponent/coefficient distributions); molecules are redrawn until
  the electron count is even and the function count lies in [10, 120].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ELEMENT_Z = {"H": 1, "He": 2, "C": 6, "N": 7, "O": 8}


def _ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


@dataclasses.dataclass
class Molecule:
    """Atoms plus a contracted Cartesian Gaussian basis, as plain arrays."""

    Z: np.ndarray            # int32 [n_atoms]
    xyz: np.ndarray          # float64 [n_atoms, 3], bohr
    shell_atom: np.ndarray   # int32 [n_shells]
    shell_l: np.ndarray      # int32 [n_shells], 0..2
    shell_nprim: np.ndarray  # int32 [n_shells]
    exps: np.ndarray         # float64 [sum(nprim)]
    coefs: np.ndarray        # float64 [sum(nprim)]
    charge: int = 0
    name: str = ""

    @property
    def n_atoms(self) -> int:
        return int(self.Z.shape[0])

    @property
    def n_shells(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def n_bf(self) -> int:
        return int(sum(_ncart(int(l)) for l in self.shell_l))

    @property
    def n_electrons(self) -> int:
        return int(self.Z.sum()) - int(self.charge)

    def shell_offsets(self) -> np.ndarray:
        """Offset of each shell's first primitive in ``exps``/``coefs``."""
        return np.concatenate([[0], np.cumsum(self.shell_nprim)[:-1]]).astype(np.int64)

    def bf_offsets(self) -> np.ndarray:
        """Index of each shell's first basis function."""
        n = [_ncart(int(l)) for l in self.shell_l]
        return np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)

    def copy(self) -> "Molecule":
        return dataclasses.replace(
            self,
            Z=self.Z.copy(), xyz=self.xyz.copy(), shell_atom=self.shell_atom.copy(),
            shell_l=self.shell_l.copy(), shell_nprim=self.shell_nprim.copy(),
            exps=self.exps.copy(), coefs=self.coefs.copy())

    def as_dict(self) -> dict:
        return {f.name: getattr(self, f.name) for f in dataclasses.fields(self)}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))


def _unit_interval_open_left(rng, n):
    # uniform in (0, 1]
    return 1.0 - rng.random(n)


def _place_points(rng, n, box, min_sep, max_tries=20000):
    """Sequential rejection sampling of n points in [0, box]^3."""
    for _restart in range(1000):
        pts = []
        tries = 0
        while len(pts) < n and tries < max_tries:
            tries += 1
            p = rng.uniform(0.0, box, size=3)
            if all(np.linalg.norm(p - q) >= min_sep for q in pts):
                pts.append(p)
        if len(pts) == n:
            return np.array(pts, dtype=np.float64)
    raise RuntimeError("could not place points")


def _assemble(Z, xyz, shells, name, charge=0) -> Molecule:
    """shells: list of (atom, l, exps array, coefs array)."""
    shell_atom = np.array([s[0] for s in shells], dtype=np.int32)
    shell_l = np.array([s[1] for s in shells], dtype=np.int32)
    shell_nprim = np.array([len(s[2]) for s in shells], dtype=np.int32)
    exps = np.concatenate([s[2] for s in shells]).astype(np.float64)
    coefs = np.concatenate([s[3] for s in shells]).astype(np.float64)
    return Molecule(np.asarray(Z, dtype=np.int32), np.asarray(xyz, dtype=np.float64),
                    shell_atom, shell_l, shell_nprim, exps, coefs, charge, name)


def random_small_molecule(seed: int, n_atoms: int = 6, elements=("H", "C", "O"),
                          box: float = 6.0, min_sep: float = 1.8,
                          shell_ls=(0, 0, 1), nprim: int = 3,
                          alpha_range=(0.1, 50.0)) -> Molecule:
    """The ``hco6_sp`` workload (defaults): random atoms, per-atom random shells."""
    rng = _rng(seed)
    while True:
        zs = np.array([ELEMENT_Z[e] for e in rng.choice(list(elements), size=n_atoms)],
                      dtype=np.int32)
        if zs.sum() % 2 == 0:
            break
    xyz = _place_points(rng, n_atoms, box, min_sep)
    shells = []
    for a in range(n_atoms):
        for l in shell_ls:
            shells.append((a, l, _log_uniform(rng, *alpha_range, nprim),
                           _unit_interval_open_left(rng, nprim)))
    return _assemble(zs, xyz, shells, f"hco6_sp/seed{seed}")


def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water_cluster(seed: int, n_waters: int = 20, box: float = 18.0,
                  min_oo: float = 5.0, min_inter: float = 1.8,
                  r_oh: float = 1.81, angle_deg: float = 104.5,
                  nprim_range=(3, 6), alpha_range=(0.05, 5000.0)) -> Molecule:
    """The ``water60_spd`` workload (defaults)."""
    rng = _rng(seed)
    half = math.radians(angle_deg) / 2.0
    local = np.array([[0.0, 0.0, 0.0],
                      [r_oh * math.sin(half), r_oh * math.cos(half), 0.0],
                      [-r_oh * math.sin(half), r_oh * math.cos(half), 0.0]])
    for _restart in range(1000):
        mols = []
        tries = 0
        while len(mols) < n_waters and tries < 200000:
            tries += 1
            o = rng.uniform(0.0, box, size=3)
            atoms = o + local @ _random_rotation(rng).T
            ok = True
            for m in mols:
                if np.linalg.norm(m[0] - o) < min_oo:
                    ok = False
                    break
                d = np.linalg.norm(m[:, None, :] - atoms[None, :, :], axis=-1)
                if d.min() < min_inter:
                    ok = False
                    break
            if ok:
                mols.append(atoms)
        if len(mols) == n_waters:
            break
    else:
        raise RuntimeError("could not place waters")
    xyz = np.concatenate(mols, axis=0)
    Z = np.array([8, 1, 1] * n_waters, dtype=np.int32)
    shells = []
    for a, z in enumerate(Z):
        ls = (0, 0, 1, 2) if z == 8 else (0, 0)
        for l in ls:
            k = int(rng.integers(nprim_range[0], nprim_range[1] + 1))
            shells.append((a, l, _log_uniform(rng, *alpha_range, k),
                           _unit_interval_open_left(rng, k)))
    return _assemble(Z, xyz, shells, f"water60_spd/seed{seed}")


_ELEMENT_SHELLS = {"H": (0, 0), "C": (0, 0, 1), "N": (0, 0, 1), "O": (0, 0, 1, 2)}


def fixed_element_basis(seed: int = 7, nprim_range=(3, 6),
                        alpha_range=(0.05, 5000.0)) -> dict:
    """One basis per element: {symbol: [(l, exps, coefs), ...]}."""
    rng = _rng(seed)
    basis = {}
    for sym in ("H", "C", "N", "O"):
        shells = []
        for l in _ELEMENT_SHELLS[sym]:
            k = int(rng.integers(nprim_range[0], nprim_range[1] + 1))
            shells.append((l, _log_uniform(rng, *alpha_range, k),
                           _unit_interval_open_left(rng, k)))
        basis[sym] = shells
    return basis


_FIXED_BASIS_CACHE: dict = {}


def batched_molecule(seed: int, n_atoms_range=(3, 20), elements=("H", "C", "N", "O"),
                     min_sep: float = 1.8, nbf_range=(10, 120),
                     basis_seed: int = 7) -> Molecule:
    """One ``mol3to20_spd`` molecule."""
    if basis_seed not in _FIXED_BASIS_CACHE:
        _FIXED_BASIS_CACHE[basis_seed] = fixed_element_basis(basis_seed)
    basis = _FIXED_BASIS_CACHE[basis_seed]
    rng = _rng(seed)
    while True:
        n = int(rng.integers(n_atoms_range[0], n_atoms_range[1] + 1))
        syms = list(rng.choice(list(elements), size=n))
        zs = np.array([ELEMENT_Z[s] for s in syms], dtype=np.int32)
        nbf = sum(_ncart(l) for s in syms for l in _ELEMENT_SHELLS[s])
        if zs.sum() % 2 == 0 and nbf_range[0] <= nbf <= nbf_range[1]:
            break
    box = 6.0 * (n / 6.0) ** (1.0 / 3.0)
    xyz = _place_points(rng, n, box, min_sep)
    shells = []
    for a, s in enumerate(syms):
        for (l, e, c) in basis[s]:
            shells.append((a, l, e.copy(), c.copy()))
    return _assemble(zs, xyz, shells, f"mol3to20_spd/seed{seed}")


def batch_of_molecules(count: int = 1024, first_seed: int = 1000) -> list:
    return [batched_molecule(first_seed + i) for i in range(count)]


def single_gaussian_system(kind: str, alpha: float, bond: float = 1.4) -> Molecule:
    """Tiny one-primitive-per-atom systems with textbook closed forms.

    kind: 'H' (one atom, 1 electron is odd: charge 0 kept, used for 1e checks),
    'He' (2 electrons), 'H2' (two H atoms `bond` bohr apart on the z axis).
    """
    if kind == "H":
        Z, xyz = [1], [[0.0, 0.0, 0.0]]
    elif kind == "He":
        Z, xyz = [2], [[0.0, 0.0, 0.0]]
    elif kind == "H2":
        Z, xyz = [1, 1], [[0.0, 0.0, 0.0], [0.0, 0.0, bond]]
    else:
        raise ValueError(kind)
    shells = [(a, 0, np.array([alpha]), np.array([1.0])) for a in range(len(Z))]
    return _assemble(Z, xyz, shells, f"{kind}/alpha{alpha}")


def conformer_scan(base: Molecule, atom: int, direction, displacements) -> list:
    """Copies of a molecule with one atom moved along a direction (bohr),
    one per displacement: the conformations of a bond scan."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    out = []
    for k, t in enumerate(displacements):
        m = base.copy()
        m.xyz = np.array(base.xyz, dtype=np.float64)
        m.xyz[atom] = m.xyz[atom] + t * d
        m.name = f"{base.name}/scan{k}"
        out.append(m)
    return out


def h2_scan(alpha: float = 0.5, count: int = 64, r_min: float = 0.6, r_max: float = 10.0) -> list:
    """Minimal-basis H2 (one s Gaussian per atom) at count bond lengths
    spaced evenly in [r_min, r_max] bohr."""
    return [single_gaussian_system("H2", alpha, bond=float(r)) for r in np.linspace(r_min, r_max, count)]


WORKLOADS = {
    "hco6_sp": random_small_molecule,
    "water60_spd": water_cluster,
    "mol3to20_spd": batched_molecule,
}


def workload(name: str, seed: int = 0) -> Molecule:
    return WORKLOADS[name](seed)


# ---------------------------------------------------------------- learned guess

MLP_SHAPES = ((256, 64), (256,), (256, 256), (256,), (128, 256), (128,))
MLP_NPARAM = sum(int(np.prod(s)) for s in MLP_SHAPES)  # 115,328


def mlp_initial_params(seed: int = 0) -> np.ndarray:
    """Initial parameters of the 64 -> 256 -> 256 -> 128 perceptron, flat
    float32 in the order W1 [256][64], b1, W2 [256][256], b2, W3 [128][256],
    b3: weights uniform in +-sqrt(6 / (fan_in + fan_out)), biases zero."""
    rng = _rng(seed)
    out = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            lim = math.sqrt(6.0 / (shape[0] + shape[1]))
            out.append(rng.uniform(-lim, lim, size=shape).astype(np.float32).ravel())
        else:
            out.append(np.zeros(shape, np.float32))
    return np.concatenate(out)


def guess_train_seeds():
    """Training, validation and test molecule seeds of the learned guess."""
    return range(100000, 110000), range(110000, 110500), range(1000, 2024)


# ---------------------------------------------------------------- densities

def symmetric_density(n: int, seed: int = 0) -> np.ndarray:
    """A seeded symmetric N x N test density: (A + A^T)/2 with A standard
    normal (PCG64(seed)).  Not a physical density; J/K are linear in D."""
    rng = _rng(seed)
    A = rng.normal(size=(n, n))
    return (A + A.T) / 2
