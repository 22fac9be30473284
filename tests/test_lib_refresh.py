"""Argument checks of the re-setup entry points that return before any
device access (CPU only): msp_refresh on a host-only context or with null
values, msp_fv_assemble_device on an operator created without a device."""
import ctypes

import numpy as np
import pytest

from gen import make_problem


def test_refresh_needs_a_device_setup_and_values():
    from paper_2407_05930_amd import Solver
    from paper_2407_05930_amd._lib import lib
    p = make_problem((12, 10, 8), s=2, seed=5)
    sv = Solver(p.A, p.img, device=-1, coarse_max=32)
    assert lib.msp_refresh(sv._ctx, None, None) == -1
    assert lib.msp_refresh(sv._ctx, ctypes.c_void_p(16), None) == -1
    assert "device" in lib.msp_last_error().decode()
    assert lib.msp_refresh(None, ctypes.c_void_p(16), None) == -1


def test_device_assembly_needs_an_operator_with_a_device():
    from paper_2407_05930_amd._lib import lib
    from paper_2407_05930_amd.adjoint import FVOperator
    pr = make_problem((10, 8, 6), s=3, seed=6, kappa="lognormal")
    op = FVOperator(pr.faces, pr.img, device=-1)
    assert op.nnz() == pr.A.nnz
    assert lib.msp_fv_assemble_device(op._h, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == -1
    assert lib.msp_fv_assemble_device(None, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == -1
    A = op.assemble(pr.kappa_base)
    assert np.array_equal(A.indptr, pr.A.indptr) and np.array_equal(A.indices, pr.A.indices)
    op.close()


def test_resetup_mode_is_validated():
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem((8, 8, 6), s=3, seed=7, kappa="lognormal")
    with pytest.raises(ValueError):
        DifferentiablePoisson(pr.faces, pr.img, device=-1, resetup="sometimes")
