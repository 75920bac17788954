"""CPU checks of the HIP library: it loads, exports every entry point the
header declares, and its host-side FP64 lattice logic (Sec. 2.1-2.2, 4.1,
4.2) agrees with the oracle.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ncl():
    from paper_1412_3784_amd import nemdcl
    return nemdcl


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "nemdcl.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(ncl_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol(ncl):
    syms = header_symbols()
    assert len(syms) >= 24
    lib = ctypes.CDLL(ncl.LIB_PATH)
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(ncl.EXPORTED) == syms


@pytest.mark.parametrize("flow", ["planar", "uniaxial", "biaxial", "shear", "none"])
def test_reduced_lattice_matches_oracle(ncl, orc, flow):
    box = wl.make_box(flow, 0.37, 100, side=12.0)
    h = ncl.ncl_create(0, 0)
    try:
        for t in np.linspace(0.0, 4.0 * (box.period or 1.0), 29):
            ncl.ncl_set_lattice(h, box.L0, box.A, t, box.automorphisms)
            L, M, c = ncl.ncl_get_lattice(h)
            Lo, Mo, co = orc.reduce(box.L0, box.A, t, box.automorphisms)
            assert np.allclose(L, Lo, rtol=0, atol=1e-13 * np.abs(Lo).max())
            if abs(abs(np.asarray(c) - np.asarray(co)).sum()) == 0:
                assert (M == Mo).all()
            else:  # a remap tie (alpha = k + 1/2): both bases are valid
                K = np.linalg.solve(L, Lo)
                assert np.allclose(K, np.round(K), atol=1e-8)
            for var, fn in (("ds", orc.ds_counts), ("do", orc.do_counts)):
                want = fn(L, 1.5)
                if want.min() >= 1:
                    ncl.ncl_set_potential(h, 1.0, 1.0, 1.5, 1)
                    got = ncl.ncl_cell_counts(h, ncl.VARIANTS[var])
                    assert list(got) == list(want)
    finally:
        ncl.ncl_destroy(h)


def test_error_codes(ncl):
    box = wl.make_box("uniaxial", 0.5, 10, side=6.0)
    h = ncl.ncl_create(0, 0)
    try:
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_set_lattice(h, box.L0, box.A, 0.3, [2 * np.eye(3, dtype=np.int32)])
        assert e.value.code == ncl.NCL_E_LATTICE
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_set_lattice(h, box.L0, box.A, 0.3, [wl.KR_M])
        assert e.value.code == ncl.NCL_E_LATTICE
        A = box.A.copy()
        A[0, 1] = 0.2
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_set_lattice(h, box.L0, A, 0.3, box.automorphisms)
        assert e.value.code == ncl.NCL_E_LATTICE
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_get_lattice(h)
        assert e.value.code == ncl.NCL_E_STATE
        ncl.ncl_set_lattice(h, box.L0, box.A, 0.3, box.automorphisms)
        ncl.ncl_set_potential(h, 1.0, 1.0, 4.0, 1)  # box side 6 < 4 cells of ... c = floor(h/4) = 1
        assert ncl.ncl_cell_counts(h, 0).min() >= 1
        ncl.ncl_set_potential(h, 1.0, 1.0, 7.0, 1)  # cut-off above every height
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_cell_counts(h, 0)
        assert e.value.code == ncl.NCL_E_BOX_TOO_SMALL
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_cell_counts(h, 5)
        assert e.value.code == ncl.NCL_E_ARG
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_set_potential(h, -1.0, 1.0, 1.0, 1)
        assert e.value.code == ncl.NCL_E_ARG
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_set_option(h, 99, 1.0)
        assert e.value.code == ncl.NCL_E_ARG
        # sweep schedules 0..3 (3: half list) and the determinism switch
        for v in (0, 1, 2, 3):
            ncl.ncl_set_option(h, ncl.NCL_OPT_SWEEP, v)
        for opt, v in ((ncl.NCL_OPT_SWEEP, 4), (ncl.NCL_OPT_DETERMINISTIC, 2)):
            with pytest.raises(ncl.NclError) as e:
                ncl.ncl_set_option(h, opt, v)
            assert e.value.code == ncl.NCL_E_ARG
        ncl.ncl_set_option(h, ncl.NCL_OPT_DETERMINISTIC, 0)
        ncl.ncl_set_option(h, ncl.NCL_OPT_DETERMINISTIC, 1)
        ncl.ncl_set_option(h, ncl.NCL_OPT_SWEEP, ncl.NCL_SWEEP_AUTO)
        # forces before any build
        with pytest.raises(ncl.NclError) as e:
            ncl._check(h, ncl._lib.ncl_compute_forces(h, None, None, None))
        assert e.value.code == ncl.NCL_E_STATE
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_get_stats(h)
        assert e.value.code == ncl.NCL_E_STATE
    finally:
        ncl.ncl_destroy(h)
    assert ncl._lib.ncl_destroy(None) == ncl.NCL_E_ARG


def test_shear_without_reset_and_rejected_flows(ncl):
    """A shear flow without automorphism is the plain L_t = (I + tA) L0; a
    non-diagonal flow that is not a shear of the lattice is rejected."""
    box = wl.make_box("shear", 0.4, 10, side=5.0, t=0.0)
    h = ncl.ncl_create(0, 0)
    try:
        ncl.ncl_set_lattice(h, box.L0, box.A, 2.5, [])
        L, M, c = ncl.ncl_get_lattice(h)
        assert np.allclose(L, (np.eye(3) + 2.5 * box.A) @ box.L0, rtol=0, atol=1e-13)
        assert (M == np.eye(3)).all()
        A = box.A.copy()
        A[1, 0] = 0.3  # A^2 != 0
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_set_lattice(h, box.L0, A, 1.0, box.automorphisms)
        assert e.value.code == ncl.NCL_E_LATTICE
        A = np.zeros((3, 3))
        A[0, 2] = 0.3  # nilpotent, but not along the automorphism's N
        with pytest.raises(ncl.NclError) as e:
            ncl.ncl_set_lattice(h, box.L0, A, 1.0, box.automorphisms)
        assert e.value.code == ncl.NCL_E_LATTICE
    finally:
        ncl.ncl_destroy(h)

