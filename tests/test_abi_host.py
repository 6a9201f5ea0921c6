"""CPU checks of libqsw: it loads, exports every function include/qsw.h
declares, and its host-only logic (theta_m, parameter selection) agrees with
the oracle's independent implementation."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2003_02450_amd as qsw
from paper_2003_02450_amd import _lib
from oracle import expmv as oexpmv
from oracle import theta as otheta

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "qsw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsw_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = _lib.load()
    declared = _declared_functions()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(_lib.EXPORTED)


def test_library_leaves_no_internal_symbol_undefined():
    """Every internal function the library calls is defined in it (a shared
    object would otherwise build and fail only when the call is reached)."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--undefined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    assert "_ZN3qsw" not in out, [ln for ln in out.splitlines() if "_ZN3qsw" in ln]


def test_status_strings_and_version():
    L = _lib.load()
    for code in range(8):
        assert L.qsw_status_str(code)
    assert b"gfx950" in L.qsw_version()


def test_library_theta_matches_oracle():
    for m in range(1, 56):
        a = qsw.theta(m)
        b = otheta.theta(m)
        assert abs(a - b) <= 1e-12 * b, (m, a, b)


def test_library_theta_single_matches_oracle():
    for m in (1, 5, 10, 20, 30, 40, 55):
        a = qsw.theta(m, single=True)
        b = otheta.theta(m, otheta.TOL_SINGLE)
        assert abs(a - b) <= 1e-12 * b, (m, a, b)


def test_theta_bad_arguments():
    L = _lib.load()
    assert L.qsw_theta(0, 0) < 0
    assert L.qsw_theta(56, 0) < 0
    assert L.qsw_theta(5, 7) < 0


def test_select_params_matches_oracle_norm1_rule():
    for x in np.concatenate([np.geomspace(1e-6, 63.0, 60), [0.0]]):
        assert qsw.select_params(x, None, 1.0) == oexpmv.select_params_norm1(x), x


def test_select_params_matches_oracle_full_rule():
    rng = np.random.Generator(np.random.PCG64(8))
    for _ in range(400):
        nrm = float(10 ** rng.uniform(-1, 2))
        d = {p: nrm * float(rng.uniform(0.01, 1.0)) for p in range(2, 10)}
        t = float(10 ** rng.uniform(-2, 3))
        n0 = int(rng.integers(1, 5))
        got = qsw.select_params(nrm, d, t, n0)
        want = oexpmv.select_params(nrm, d, t, n0)
        assert got == want, (nrm, t, n0, got, want)


def test_select_params_rejects_bad_input():
    with pytest.raises(qsw.QswError):
        qsw.select_params(float("nan"), None, 1.0)
    with pytest.raises(qsw.QswError):
        qsw.select_params(1.0, None, float("inf"))


def test_select_params_fp32_matches_oracle_capped_rule():
    """QSW_PREC_FP32: the single-precision theta_m with m <= 20, p <= 5."""
    th = otheta.theta_table(otheta.TOL_SINGLE)
    rng = np.random.Generator(np.random.PCG64(9))
    for _ in range(300):
        nrm = float(10 ** rng.uniform(-1, 2))
        d = {p: nrm * float(rng.uniform(0.01, 1.0)) for p in range(2, 10)}
        t = float(10 ** rng.uniform(-2, 3))
        n0 = int(rng.integers(1, 5))
        got = qsw.select_params(nrm, d, t, n0, single="fp32")
        want = oexpmv.select_params(nrm, d, t, n0, thetas=th, m_max=20, p_max=5)
        assert got == want, (nrm, t, n0, got, want)
        assert got[0] <= 20


def test_select_params_known_norms_matches_oracle_without_switch():
    """QSW_PARAMS_KNOWN_NORMS (the rule propagate uses with a handle's norms):
    the alpha_p rule at every ||tL||_1, as the oracle's rule without the
    condition-3.13 switch; for large ||tL||_1 it is the published rule."""
    rng = np.random.Generator(np.random.PCG64(10))
    for prec, th, mm, pm in (("double", otheta.theta_table(), 55, 8),
                             ("fp32", otheta.theta_table(otheta.TOL_SINGLE), 20, 5)):
        for _ in range(300):
            nrm = float(10 ** rng.uniform(-1, 2))
            d = {p: nrm * float(rng.uniform(0.01, 1.0)) for p in range(2, 10)}
            t = float(10 ** rng.uniform(-3, 3))
            n0 = int(rng.integers(1, 5))
            got = qsw.select_params(nrm, d, t, n0, single=prec, known_norms=True)
            want = oexpmv.select_params(nrm, d, t, n0, thetas=th, m_max=mm, p_max=pm,
                                        switch=False)
            assert got == want, (prec, nrm, t, n0, got, want)
            if not oexpmv.condition_3_13(t * nrm, n0, thetas=th, m_max=mm, p_max=pm):
                assert got == qsw.select_params(nrm, d, t, n0, single=prec)

