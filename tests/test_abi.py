"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/mess.h declares, and argument validation returns the
documented status codes before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mess.h")


@pytest.fixture(scope="module")
def mess():
    from paper_2406_03121_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build()
    from paper_2406_03121_amd import mess as m
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mess_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(mess):
    names = declared_functions()
    assert len(names) >= 15
    L = mess.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(mess.EXPORTED)


def _basis_args(l=(0, 1), nprim=(2, 1), exps=(1.0, 0.5, 0.3), atom=(0, 0)):
    Z = np.array([8], np.int32)
    xyz = np.zeros(3)
    sl = np.array(l, np.int32)
    sn = np.array(nprim, np.int32)
    sa = np.array(atom, np.int32)
    ex = np.array(exps, np.float64)
    co = np.ones(len(exps))
    return Z, xyz, sa, sl, sn, ex, co


def _create(mess, args, charge=0):
    Z, xyz, sa, sl, sn, ex, co = args
    h = ctypes.c_void_p()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    rc = mess.lib().mess_basis_create(len(Z), p(Z), p(xyz), len(sl), p(sa), p(sl), p(sn), p(ex), p(co), charge,
                                      ctypes.byref(h))
    return rc, h


def test_basis_create_validation(mess):
    rc, _ = _create(mess, _basis_args(l=(0, 3)))
    assert rc == mess.MESS_E_UNSUPPORTED and "l=3" in mess.mess_last_error()
    rc, _ = _create(mess, _basis_args(exps=(1.0, -0.5, 0.3)))
    assert rc == mess.MESS_E_ARG and "exponent" in mess.mess_last_error()
    rc, _ = _create(mess, _basis_args(exps=(1.0, float("nan"), 0.3)))
    assert rc == mess.MESS_E_ARG
    rc, _ = _create(mess, _basis_args(atom=(0, 1)))
    assert rc == mess.MESS_E_ARG and "atom" in mess.mess_last_error()
    rc, _ = _create(mess, _basis_args(nprim=(0, 3)))
    assert rc == mess.MESS_E_ARG
    rc, _ = _create(mess, _basis_args(l=(0, -1)))
    assert rc == mess.MESS_E_ARG
    Z, xyz, sa, sl, sn, ex, co = _basis_args()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    assert mess.lib().mess_basis_create(1, p(Z), p(xyz), 2, p(sa), p(sl), p(sn), p(ex), p(co), 0, None) == \
        mess.MESS_E_ARG


def test_null_handles(mess):
    L = mess.lib()
    L.mess_basis_destroy(None)
    L.mess_scf_destroy(None)
    assert L.mess_basis_info(None, None, None, None) == mess.MESS_E_ARG
    assert L.mess_jk(None, None, None, None, 0, 0, 0.0, None) == mess.MESS_E_ARG
    assert L.mess_eri(None, 0, 0, 0.0, None, 0, None) == mess.MESS_E_ARG
    assert L.mess_one_electron(None, None, None, None, None) == mess.MESS_E_ARG
    assert L.mess_scf_create(None, None, None, None) == mess.MESS_E_ARG
    assert L.mess_scf_step(None, None, None, None, None, None) == mess.MESS_E_ARG
    assert L.mess_scf_density(None, None, None) == mess.MESS_E_ARG
    assert mess.mess_last_error() != ""


def test_work_stats_rejects_bad_class(mess):
    L = mess.lib()
    assert L.mess_work_stats(None, 0.0, 0, None, None, None) == mess.MESS_E_ARG


def test_kernel_form_table(mess):
    """The form table is host state: validation needs no device."""
    L = mess.lib()
    act = ctypes.c_int32()
    assert L.mess_kernel_form(0, 21, -1, ctypes.byref(act)) == mess.MESS_E_ARG
    assert L.mess_kernel_form(0, -1, -1, None) == mess.MESS_E_ARG
    assert L.mess_kernel_form(9, 0, -1, None) == mess.MESS_E_ARG
    # (ss|ss) has no primitive-lane or table-driven form
    assert L.mess_kernel_form(0, 0, mess.MESS_FORM_PLANE, None) == mess.MESS_E_UNSUPPORTED
    # forms are kept per precision
    assert mess.mess_kernel_form(0, mess.MESS_FORM_LANE, prec=mess.MESS_FP32) == mess.MESS_FORM_LANE
    assert mess.mess_kernel_form(0) == mess.MESS_FORM_ROWS
    # FP32 builds run (ss|ss) with its FP64 kernel by default
    assert mess.mess_kernel_form(0, mess.MESS_FORM_AUTO, prec=mess.MESS_FP32) == mess.MESS_FORM_FP64
    assert L.mess_kernel_form(0, 0, mess.MESS_FORM_FP64, None) == mess.MESS_E_UNSUPPORTED
    assert mess.mess_kernel_form(mess.class_index(5, 5), prec=mess.MESS_FP32) == mess.MESS_FORM_WAVE
    assert mess.mess_kernel_form(0) == mess.MESS_FORM_ROWS          # built-in default
    assert mess.mess_kernel_form(0, mess.MESS_FORM_LANE) == mess.MESS_FORM_LANE
    assert mess.mess_kernel_form(0, mess.MESS_FORM_AUTO) == mess.MESS_FORM_ROWS
    dd_dd = mess.class_index(5, 5)
    assert mess.mess_kernel_form(dd_dd) == mess.MESS_FORM_WAVE
    assert L.mess_kernel_form(0, dd_dd, mess.MESS_FORM_LANE, None) == mess.MESS_E_UNSUPPORTED
    dd_dp = mess.class_index(5, 4)
    assert mess.mess_kernel_form(dd_dp) == mess.MESS_FORM_PLANE


def test_new_entry_points_reject_null(mess):
    L = mess.lib()
    assert L.mess_autotune(None, 0, 0.0, None, 1, None, None, None) == mess.MESS_E_ARG
    assert L.mess_eri_quartets(None, 0.0, None, None) == mess.MESS_E_ARG
    assert L.mess_jk_noalloc(None, None, None, None, 0, 0.0, None) == mess.MESS_E_ARG
    assert L.mess_jk(None, None, None, None, mess.MESS_JK_DETERMINISTIC, 0, 0.0, None) == mess.MESS_E_ARG
