"""Thin ctypes binding of libmess_hip.so (argument marshalling only).

Every function here forwards to the C entry point of the same name declared
in include/mess.h.  Matrices are torch tensors on a HIP device (float64,
contiguous, row-major); atom and shell arrays are host numpy arrays.  There
is no fallback: if the library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmess_hip.so")

MESS_OK, MESS_E_ARG, MESS_E_UNSUPPORTED, MESS_E_NOMEM, MESS_E_DEVICE, MESS_E_NUMERIC, MESS_E_SIZE = range(7)
MESS_FP64, MESS_FP32 = 0, 1
MESS_ERI_DENSE, MESS_ERI_BLOCKS = 0, 1
MESS_JK_DIRECT, MESS_JK_STORED, MESS_JK_DETERMINISTIC = 0, 1, 2
MESS_XC_HF, MESS_XC_LDA_X, MESS_XC_PBE = 0, 1, 2
MESS_FORM_AUTO, MESS_FORM_LANE, MESS_FORM_ROWS, MESS_FORM_PLANE, MESS_FORM_COOP, MESS_FORM_WAVE, MESS_FORM_FP64 = range(7)

EXPORTED = [
    "mess_basis_create", "mess_basis_destroy", "mess_basis_info", "mess_one_electron",
    "mess_eri", "mess_jk", "mess_scf_create", "mess_scf_step", "mess_scf_density",
    "mess_scf_fock", "mess_scf_destroy", "mess_last_error",
    "mess_work_stats", "mess_prim_pairs", "mess_prof_enable", "mess_prof_read",
    "mess_batch_create", "mess_batch_info", "mess_batch_scf_create", "mess_batch_scf_step",
    "mess_batch_scf_status", "mess_batch_scf_density", "mess_batch_scf_destroy",
    "mess_lda_x", "mess_pbe_xc", "mess_grid",
    "mess_mlp_create", "mess_mlp_destroy", "mess_mlp_params", "mess_mlp_forward", "mess_mlp_grad",
    "mess_mlp_train_step", "mess_guess_rows", "mess_guess_features", "mess_guess_targets",
    "mess_guess_assemble", "mess_guess_project", "mess_guess_judge",
    "mess_kernel_form", "mess_autotune", "mess_hf_gradient", "mess_scf_gradient", "mess_scf_guard", "mess_batch_scf_guard", "mess_jk_noalloc", "mess_jk_dense", "mess_eri_quartets", "mess_boys", "mess_dmin_step",
    "mess_dmin_trial", "mess_dmin_eval",
]
MESS_MLP_NPARAM = 115328


class MessError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where} -> status {code}: {msg}")
        self.code = code


class ScfOpts(ctypes.Structure):
    _fields_ = [("schwarz_tol", ctypes.c_double), ("conv_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("diis_size", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("jk_mode", ctypes.c_int32),
                ("xc", ctypes.c_int32), ("deterministic", ctypes.c_int32), ("no_guard", ctypes.c_int32)]


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built; run `python -m paper_2406_03121_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        L.mess_basis_create.argtypes = [i32, vp, vp, i32, vp, vp, vp, vp, vp, i32, ctypes.POINTER(vp)]
        L.mess_basis_destroy.argtypes = [vp]
        L.mess_basis_destroy.restype = None
        L.mess_basis_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(f64)]
        L.mess_one_electron.argtypes = [vp, vp, vp, vp, vp]
        L.mess_eri.argtypes = [vp, i32, i32, f64, vp, sz, vp]
        L.mess_jk.argtypes = [vp, vp, vp, vp, i32, i32, f64, vp]
        L.mess_jk_noalloc.argtypes = [vp, vp, vp, vp, i32, f64, vp]
        L.mess_eri_quartets.argtypes = [vp, f64, vp, vp]
        L.mess_boys.argtypes = [vp, i32, i32, i32, vp, ctypes.c_int64, vp, vp]
        L.mess_jk_dense.argtypes = [vp, i32, i32, vp, vp, vp, i32, i32, vp]
        L.mess_dmin_step.argtypes = [vp, f64, ctypes.POINTER(f64), ctypes.POINTER(f64), vp]
        L.mess_dmin_trial.argtypes = [vp, vp, vp]
        L.mess_dmin_eval.argtypes = [vp, vp, ctypes.POINTER(f64), vp, vp]
        if hasattr(L, "mess_scf_create"):
            L.mess_scf_create.argtypes = [vp, ctypes.POINTER(ScfOpts), vp, ctypes.POINTER(vp)]
            L.mess_scf_step.argtypes = [vp, ctypes.POINTER(f64), ctypes.POINTER(f64), ctypes.POINTER(f64),
                                        ctypes.POINTER(i32), vp]
            L.mess_scf_density.argtypes = [vp, vp, vp]
            L.mess_scf_fock.argtypes = [vp, vp, vp]
            L.mess_scf_destroy.argtypes = [vp]
            L.mess_scf_destroy.restype = None
            L.mess_scf_guard.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
            L.mess_hf_gradient.argtypes = [vp, vp, vp, f64, vp, vp]
            L.mess_scf_gradient.argtypes = [vp, vp, vp]
            L.mess_batch_scf_guard.argtypes = [vp, vp]
        i64 = ctypes.c_int64
        f32 = ctypes.c_float
        L.mess_mlp_create.argtypes = [vp, ctypes.POINTER(vp)]
        L.mess_mlp_destroy.argtypes = [vp]
        L.mess_mlp_destroy.restype = None
        L.mess_mlp_params.argtypes = [vp, vp]
        L.mess_mlp_forward.argtypes = [vp, i64, vp, vp, vp]
        L.mess_mlp_grad.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.POINTER(f64), vp]
        L.mess_mlp_train_step.argtypes = [vp, i64, vp, vp, vp, f32, ctypes.POINTER(f64), vp]
        L.mess_guess_rows.argtypes = [vp, ctypes.POINTER(i64)]
        L.mess_guess_features.argtypes = [vp, vp, vp]
        L.mess_guess_targets.argtypes = [vp, vp, vp, vp, vp]
        L.mess_guess_assemble.argtypes = [vp, vp, vp, vp]
        L.mess_guess_project.argtypes = [vp, vp, vp]
        L.mess_guess_judge.argtypes = [vp, ctypes.POINTER(ScfOpts), vp, vp, vp]
        L.mess_lda_x.argtypes = [vp, vp, vp, ctypes.POINTER(f64), vp, vp]
        L.mess_pbe_xc.argtypes = [vp, vp, vp, ctypes.POINTER(f64), vp, vp, vp]
        L.mess_grid.argtypes = [vp, vp, ctypes.POINTER(i64), vp]
        L.mess_batch_create.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.mess_batch_info.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mess_batch_scf_create.argtypes = [vp, ctypes.POINTER(ScfOpts), vp, i32, ctypes.POINTER(vp)]
        L.mess_batch_scf_step.argtypes = [vp, vp]
        L.mess_batch_scf_status.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.mess_batch_scf_density.argtypes = [vp, vp, vp]
        L.mess_batch_scf_destroy.argtypes = [vp]
        L.mess_batch_scf_destroy.restype = None
        L.mess_work_stats.argtypes = [vp, f64, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(f64)]
        L.mess_prim_pairs.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.mess_prof_enable.argtypes = [i32]
        L.mess_prof_read.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(f64), ctypes.POINTER(f64),
                                     ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.mess_kernel_form.argtypes = [i32, i32, i32, ctypes.POINTER(i32)]
        L.mess_autotune.argtypes = [vp, i32, f64, vp, i32, vp, vp, vp]
        L.mess_last_error.argtypes = []
        L.mess_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def mess_last_error() -> str:
    return lib().mess_last_error().decode()


def _check(rc, where):
    if rc != MESS_OK:
        raise MessError(rc, where, mess_last_error())


def _ptr(t):
    """Device pointer of a torch tensor (or None -> NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Basis:
    """Owning wrapper of a mess_basis handle (one molecule or a batch).

    For a batch, mol_nbf / mol_moff / mol_nocc / mol_enuc describe the
    packed block-diagonal layout of every matrix (packed = mol_moff[-1])."""

    def __init__(self, handle):
        self.handle = handle
        nbf, nocc, enuc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().mess_basis_info(handle, ctypes.byref(nbf), ctypes.byref(nocc), ctypes.byref(enuc)),
               "mess_basis_info")
        self.nbf, self.n_occ, self.e_nuc = nbf.value, nocc.value, enuc.value
        nm = ctypes.c_int32()
        _check(lib().mess_batch_info(handle, ctypes.byref(nm), None, None, None, None), "mess_batch_info")
        self.n_mol = nm.value
        self.mol_nbf = np.zeros(self.n_mol, np.int32)
        self.mol_moff = np.zeros(self.n_mol + 1, np.int64)
        self.mol_nocc = np.zeros(self.n_mol, np.int32)
        self.mol_enuc = np.zeros(self.n_mol, np.float64)
        _check(lib().mess_batch_info(handle, None, self.mol_nbf.ctypes.data_as(ctypes.c_void_p),
                                     self.mol_moff.ctypes.data_as(ctypes.c_void_p),
                                     self.mol_nocc.ctypes.data_as(ctypes.c_void_p),
                                     self.mol_enuc.ctypes.data_as(ctypes.c_void_p)), "mess_batch_info")
        self.packed = int(self.mol_moff[-1])

    def close(self):
        if self.handle:
            lib().mess_basis_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mess_basis_create(Z, xyz, shell_atom, shell_l, shell_nprim, exps, coefs, charge=0) -> Basis:
    Z, pZ = _host(Z, np.int32)
    xyz, pX = _host(xyz, np.float64)
    sa, pA = _host(shell_atom, np.int32)
    sl, pL = _host(shell_l, np.int32)
    sn, pN = _host(shell_nprim, np.int32)
    ex, pE = _host(exps, np.float64)
    co, pC = _host(coefs, np.float64)
    h = ctypes.c_void_p()
    _check(lib().mess_basis_create(len(Z), pZ, pX, len(sl), pA, pL, pN, pE, pC, int(charge), ctypes.byref(h)),
           "mess_basis_create")
    b = Basis(h)
    b.n_atoms = len(Z)
    return b


def basis_from_molecule(mol) -> Basis:
    """Convenience: a mess_inputs.Molecule -> Basis."""
    return mess_basis_create(mol.Z, mol.xyz, mol.shell_atom, mol.shell_l, mol.shell_nprim, mol.exps,
                             mol.coefs, mol.charge)


def mess_batch_create(mols) -> Basis:
    """A batch handle over a list of mess_inputs.Molecule (per-molecule
    shell_atom indices stay local)."""
    cat = lambda f, dt: np.ascontiguousarray(np.concatenate([np.asarray(getattr(m, f)) for m in mols]), dt)  # noqa: E731
    na, pna = _host([len(m.Z) for m in mols], np.int32)
    ns, pns = _host([len(m.shell_l) for m in mols], np.int32)
    ch, pch = _host([m.charge for m in mols], np.int32)
    Z, pZ = _host(cat("Z", np.int32), np.int32)
    xyz, pX = _host(np.concatenate([np.asarray(m.xyz, np.float64).reshape(-1, 3) for m in mols]), np.float64)
    sa, pA = _host(cat("shell_atom", np.int32), np.int32)
    sl, pL = _host(cat("shell_l", np.int32), np.int32)
    sn, pN = _host(cat("shell_nprim", np.int32), np.int32)
    ex, pE = _host(cat("exps", np.float64), np.float64)
    co, pC = _host(cat("coefs", np.float64), np.float64)
    h = ctypes.c_void_p()
    _check(lib().mess_batch_create(len(mols), pna, pns, pch, pZ, pX, pA, pL, pN, pE, pC, ctypes.byref(h)),
           "mess_batch_create")
    b = Basis(h)
    b.n_atoms = len(Z)
    return b


def mess_one_electron(basis: Basis, S=None, T=None, V=None, stream=None):
    _check(lib().mess_one_electron(basis.handle, _ptr(S), _ptr(T), _ptr(V), _stream(stream)),
           "mess_one_electron")


def mess_eri(basis: Basis, out, layout=MESS_ERI_DENSE, prec=MESS_FP64, schwarz_tol=0.0, stream=None):
    nbytes = out.numel() * out.element_size()
    _check(lib().mess_eri(basis.handle, int(layout), int(prec), float(schwarz_tol), _ptr(out), nbytes,
                          _stream(stream)), "mess_eri")


def mess_eri_quartets(basis: Basis, schwarz_tol=0.0):
    """(counts[21], shells[sum counts, 4]) of the MESS_ERI_BLOCKS layout."""
    counts = np.zeros(21, np.int64)
    _check(lib().mess_eri_quartets(basis.handle, float(schwarz_tol), counts.ctypes.data_as(ctypes.c_void_p), None),
           "mess_eri_quartets")
    shells = np.zeros((max(1, int(counts.sum())), 4), np.int32)
    _check(lib().mess_eri_quartets(basis.handle, float(schwarz_tol), None, shells.ctypes.data_as(ctypes.c_void_p)),
           "mess_eri_quartets")
    return counts, shells[:int(counts.sum())]


MESS_DENSE_VALU, MESS_DENSE_MFMA = 0, 1


def mess_jk_dense(eri, n, D, J=None, K=None, prec=MESS_FP64, form=MESS_DENSE_MFMA, stream=None):
    """J, K [ndens, n, n] of the densities D [ndens, n, n] from the dense tensor eri (n^4)."""
    nd = D.numel() // (n * n)
    _check(lib().mess_jk_dense(_ptr(eri), int(n), int(nd), _ptr(D), _ptr(J), _ptr(K), int(prec), int(form),
                               _stream(stream)), "mess_jk_dense")


def mess_boys(basis: Basis, T, F, m, form=0, prec=MESS_FP64, stream=None):
    """F[i, j] = F_j(T[i]), j = 0..m, on the device (T: float64 [n], F: float64 [n, m + 1])."""
    _check(lib().mess_boys(basis.handle, int(prec), int(form), int(m), _ptr(T), int(T.numel()), _ptr(F),
                           _stream(stream)), "mess_boys")


def mess_jk(basis: Basis, D, J=None, K=None, mode=MESS_JK_DIRECT, prec=MESS_FP64, schwarz_tol=0.0,
            stream=None):
    _check(lib().mess_jk(basis.handle, _ptr(D), _ptr(J), _ptr(K), int(mode), int(prec), float(schwarz_tol),
                         _stream(stream)), "mess_jk")


def mess_jk_noalloc(basis: Basis, D, J=None, K=None, prec=MESS_FP64, schwarz_tol=0.0, stream=None):
    """Direct J/K with no device allocation (fixed library workspace); the
    work lists must exist (an earlier mess_jk on this basis and tolerance)."""
    _check(lib().mess_jk_noalloc(basis.handle, _ptr(D), _ptr(J), _ptr(K), int(prec), float(schwarz_tol),
                                 _stream(stream)), "mess_jk_noalloc")


def mess_lda_x(basis: Basis, D, Vx=None, rho=None, stream=None):
    """E_x (host float); fills Vx (N x N) and rho (grid points) if given."""
    ex = ctypes.c_double()
    _check(lib().mess_lda_x(basis.handle, _ptr(D), _ptr(Vx), ctypes.byref(ex), _ptr(rho), _stream(stream)),
           "mess_lda_x")
    return ex.value


def mess_pbe_xc(basis: Basis, D, Vxc=None, rho=None, grad_rho=None, stream=None):
    """E_xc (host float); fills Vxc (N x N), rho [npts] and grad_rho [3, npts] if given."""
    ex = ctypes.c_double()
    _check(lib().mess_pbe_xc(basis.handle, _ptr(D), _ptr(Vxc), ctypes.byref(ex), _ptr(rho), _ptr(grad_rho),
                             _stream(stream)), "mess_pbe_xc")
    return ex.value


def mess_grid(basis: Basis, xyzw=None, stream=None):
    """Number of LDA grid points; fills xyzw [npts, 4] if given."""
    n = ctypes.c_int64()
    _check(lib().mess_grid(basis.handle, _ptr(xyzw), ctypes.byref(n), _stream(stream)), "mess_grid")
    return n.value


class Scf:
    """Owning wrapper of a mess_scf handle."""

    def __init__(self, handle, basis):
        self.handle, self.basis = handle, basis

    def close(self):
        if self.handle:
            lib().mess_scf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mess_scf_create(basis: Basis, schwarz_tol=0.0, conv_tol=1e-8, max_iter=100, diis_size=8,
                    prec=MESS_FP64, jk_mode=MESS_JK_DIRECT, xc=MESS_XC_HF, D0=None, deterministic=False,
                    guard=True) -> Scf:
    opts = ScfOpts(float(schwarz_tol), float(conv_tol), int(max_iter), int(diis_size), int(prec),
                   int(jk_mode), int(xc), 1 if deterministic else 0, 0 if guard else 1)
    h = ctypes.c_void_p()
    _check(lib().mess_scf_create(basis.handle, ctypes.byref(opts), _ptr(D0), ctypes.byref(h)), "mess_scf_create")
    return Scf(h, basis)


def mess_dmin_step(scf: Scf, lr=0.1, stream=None):
    """One direct-minimisation (Adam) step; returns (energy, max |dE/dZ|)."""
    e, g = ctypes.c_double(), ctypes.c_double()
    _check(lib().mess_dmin_step(scf.handle, float(lr), ctypes.byref(e), ctypes.byref(g), _stream(stream)),
           "mess_dmin_step")
    return e.value, g.value


def mess_dmin_eval(scf: Scf, Z, G=None, stream=None):
    """E(Z) (returned) and dE/dZ into G (device N x N, optional)."""
    e = ctypes.c_double()
    _check(lib().mess_dmin_eval(scf.handle, _ptr(Z), ctypes.byref(e), _ptr(G), _stream(stream)), "mess_dmin_eval")
    return e.value


def mess_dmin_trial(scf: Scf, Z, stream=None):
    _check(lib().mess_dmin_trial(scf.handle, _ptr(Z), _stream(stream)), "mess_dmin_trial")


def mess_scf_guard(scf: Scf):
    """(stage, rises) of the divergence guard."""
    st, r = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mess_scf_guard(scf.handle, ctypes.byref(st), ctypes.byref(r)), "mess_scf_guard")
    return st.value, r.value


def mess_hf_gradient(basis: Basis, D, F, schwarz_tol=0.0, stream=None):
    """dE/dR (numpy [n_atoms, 3]) at the converged density D and Fock matrix F."""
    g = np.zeros((basis.n_atoms, 3))
    _check(lib().mess_hf_gradient(basis.handle, _ptr(D), _ptr(F), float(schwarz_tol),
                                  g.ctypes.data_as(ctypes.c_void_p), _stream(stream)), "mess_hf_gradient")
    return g


def mess_scf_gradient(scf: Scf, stream=None):
    """dE/dR (numpy [n_atoms, 3]) of a converged SCF handle."""
    g = np.zeros((scf.basis.n_atoms, 3))
    _check(lib().mess_scf_gradient(scf.handle, g.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
           "mess_scf_gradient")
    return g


def mess_batch_scf_guard(scf):
    """Per-molecule divergence-guard stages (numpy int32 [n_mol])."""
    n = scf.basis.n_mol
    st = np.zeros(max(1, n), np.int32)
    _check(lib().mess_batch_scf_guard(scf.handle, st.ctypes.data_as(ctypes.c_void_p)), "mess_batch_scf_guard")
    return st[:n]


def mess_scf_step(scf: Scf, stream=None):
    """Returns (energy, delta_e, resid, converged)."""
    e, de, r, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    _check(lib().mess_scf_step(scf.handle, ctypes.byref(e), ctypes.byref(de), ctypes.byref(r), ctypes.byref(c),
                               _stream(stream)), "mess_scf_step")
    return e.value, de.value, r.value, bool(c.value)


def mess_scf_density(scf: Scf, D, stream=None):
    _check(lib().mess_scf_density(scf.handle, _ptr(D), _stream(stream)), "mess_scf_density")


def mess_scf_fock(scf: Scf, F, stream=None):
    _check(lib().mess_scf_fock(scf.handle, _ptr(F), _stream(stream)), "mess_scf_fock")


class BatchScf:
    """Owning wrapper of a mess_batch_scf handle."""

    def __init__(self, handle, basis):
        self.handle, self.basis = handle, basis

    def close(self):
        if self.handle:
            lib().mess_batch_scf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mess_batch_scf_create(basis: Basis, schwarz_tol=0.0, conv_tol=1e-8, max_iter=100, diis_size=8,
                          jk_mode=MESS_JK_DIRECT, D0=None, use_graph=False, prec=MESS_FP64,
                          guard=True) -> BatchScf:
    opts = ScfOpts(float(schwarz_tol), float(conv_tol), int(max_iter), int(diis_size), int(prec),
                   int(jk_mode), MESS_XC_HF, 0, 0 if guard else 1)
    h = ctypes.c_void_p()
    _check(lib().mess_batch_scf_create(basis.handle, ctypes.byref(opts), _ptr(D0), 1 if use_graph else 0,
                                       ctypes.byref(h)), "mess_batch_scf_create")
    return BatchScf(h, basis)


def mess_batch_scf_step(scf: BatchScf, stream=None):
    _check(lib().mess_batch_scf_step(scf.handle, _stream(stream)), "mess_batch_scf_step")


def mess_batch_scf_status(scf: BatchScf, stream=None):
    """dict of per-molecule numpy arrays energy, delta_e, resid, converged, and n_converged."""
    n = scf.basis.n_mol
    e, de, r = np.zeros(n), np.zeros(n), np.zeros(n)
    c = np.zeros(n, np.int32)
    nc = ctypes.c_int32()
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    _check(lib().mess_batch_scf_status(scf.handle, vp(e), vp(de), vp(r), vp(c), ctypes.byref(nc),
                                       _stream(stream)), "mess_batch_scf_status")
    return {"energy": e, "delta_e": de, "resid": r, "converged": c.astype(bool), "n_converged": nc.value}


def mess_batch_scf_density(scf: BatchScf, D, stream=None):
    _check(lib().mess_batch_scf_density(scf.handle, _ptr(D), _stream(stream)), "mess_batch_scf_density")


class Mlp:
    """Owning wrapper of a mess_mlp handle (the learned-guess perceptron)."""

    def __init__(self, params):
        p = np.ascontiguousarray(params, np.float32)
        if p.size != MESS_MLP_NPARAM:
            raise ValueError(f"expected {MESS_MLP_NPARAM} parameters, got {p.size}")
        h = ctypes.c_void_p()
        _check(lib().mess_mlp_create(p.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)), "mess_mlp_create")
        self.handle = h

    def params(self):
        out = np.zeros(MESS_MLP_NPARAM, np.float32)
        _check(lib().mess_mlp_params(self.handle, out.ctypes.data_as(ctypes.c_void_p)), "mess_mlp_params")
        return out

    def forward(self, X, Y, stream=None):
        _check(lib().mess_mlp_forward(self.handle, X.shape[0], _ptr(X), _ptr(Y), _stream(stream)),
               "mess_mlp_forward")

    def grad(self, X, T, M, grad=None, stream=None):
        loss = ctypes.c_double()
        _check(lib().mess_mlp_grad(self.handle, X.shape[0], _ptr(X), _ptr(T), _ptr(M), _ptr(grad),
                                   ctypes.byref(loss), _stream(stream)), "mess_mlp_grad")
        return loss.value

    def train_step(self, X, T, M, lr=1e-3, want_loss=True, stream=None):
        loss = ctypes.c_double()
        _check(lib().mess_mlp_train_step(self.handle, X.shape[0], _ptr(X), _ptr(T), _ptr(M), float(lr),
                                         ctypes.byref(loss) if want_loss else None, _stream(stream)),
               "mess_mlp_train_step")
        return loss.value if want_loss else None

    def close(self):
        if self.handle:
            lib().mess_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mess_guess_rows(basis: Basis):
    n = ctypes.c_int64()
    _check(lib().mess_guess_rows(basis.handle, ctypes.byref(n)), "mess_guess_rows")
    return n.value


def mess_guess_features(basis: Basis, X, stream=None):
    _check(lib().mess_guess_features(basis.handle, _ptr(X), _stream(stream)), "mess_guess_features")


def mess_guess_targets(basis: Basis, D, T=None, M=None, stream=None):
    _check(lib().mess_guess_targets(basis.handle, _ptr(D), _ptr(T), _ptr(M), _stream(stream)),
           "mess_guess_targets")


def mess_guess_assemble(basis: Basis, Y, D, stream=None):
    _check(lib().mess_guess_assemble(basis.handle, _ptr(Y), _ptr(D), _stream(stream)), "mess_guess_assemble")


def mess_guess_project(basis: Basis, D, stream=None):
    _check(lib().mess_guess_project(basis.handle, _ptr(D), _stream(stream)), "mess_guess_project")


def mess_guess_judge(basis: Basis, D0, schwarz_tol=1e-10, stream=None):
    """Replaces, per molecule, D0's block by the core guess where that has the
    smaller first commutator residual; returns the per-molecule 'kept' flags."""
    opts = ScfOpts(float(schwarz_tol), 1e-8, 100, 8, MESS_FP64, MESS_JK_DIRECT, MESS_XC_HF, 0)
    used = np.zeros(basis.n_mol, np.int32)
    _check(lib().mess_guess_judge(basis.handle, ctypes.byref(opts), _ptr(D0), used.ctypes.data_as(ctypes.c_void_p),
                                  _stream(stream)), "mess_guess_judge")
    return used.astype(bool)


def class_index(cb, ck):
    return cb * (cb + 1) // 2 + ck


def mess_work_stats(basis: Basis, schwarz_tol, cls):
    """(shell quartets, primitive quartets, algorithmic FP64 ops of one J/K pass) of class cls."""
    q, p, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    _check(lib().mess_work_stats(basis.handle, float(schwarz_tol), int(cls), ctypes.byref(q), ctypes.byref(p),
                                 ctypes.byref(f)), "mess_work_stats")
    return q.value, p.value, f.value


def mess_prim_pairs(basis: Basis):
    """(primitive pairs kept by the basis's screening, primitive pairs before it)."""
    k, f = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().mess_prim_pairs(basis.handle, ctypes.byref(k), ctypes.byref(f)), "mess_prim_pairs")
    return k.value, f.value


def mess_prof_enable(on=True):
    _check(lib().mess_prof_enable(1 if on else 0), "mess_prof_enable")


def mess_prof_read(cls=-1):
    """dict(launches, ms, alg_flops, quartets, prim_quartets) for class cls (-1: all)."""
    n, q, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    ms, f = ctypes.c_double(), ctypes.c_double()
    _check(lib().mess_prof_read(int(cls), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(f), ctypes.byref(q),
                                ctypes.byref(p)), "mess_prof_read")
    return {"launches": n.value, "ms": ms.value, "alg_flops": f.value, "quartets": q.value,
            "prim_quartets": p.value}


def mess_kernel_form(cls, form=-1, prec=MESS_FP64):
    """Set the kernel form of class cls in precision prec (form >= 0);
    returns the active form."""
    act = ctypes.c_int32()
    _check(lib().mess_kernel_form(int(prec), int(cls), int(form), ctypes.byref(act)), "mess_kernel_form")
    return act.value


def mess_autotune(basis: Basis, D, schwarz_tol=0.0, reps=3, prec=MESS_FP64, stream=None):
    """Time every form of every class on the basis and keep the fastest.
    Returns (forms[21], ms[21, 7]) as numpy arrays."""
    forms = np.zeros(21, np.int32)
    ms = np.zeros(21 * 7, np.float64)
    _check(lib().mess_autotune(basis.handle, int(prec), float(schwarz_tol), _ptr(D), int(reps),
                               forms.ctypes.data_as(ctypes.c_void_p), ms.ctypes.data_as(ctypes.c_void_p),
                               _stream(stream)), "mess_autotune")
    return forms, ms.reshape(21, 7)
