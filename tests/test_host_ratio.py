"""R(t) = G_E(t) / G_0(t) (Sec. 4) computed by the library's host routine ov_ratio_R.

CPU only (the routine takes host arrays and needs no GPU): against the correlator oracle's
ratio of the mean field correlator, and the error codes for invalid correlators.
"""
import ctypes
import os

import numpy as np
import pytest

from oracle import corr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1111_6288_amd", "libov.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libov.so not built")


def _call(ge, g0):
    lib = ctypes.CDLL(LIB)
    pd = ctypes.POINTER(ctypes.c_double)
    ge = np.ascontiguousarray(ge, dtype=np.float64)
    g0 = np.ascontiguousarray(g0, dtype=np.float64)
    out = np.zeros(g0.shape[0])
    rc = lib.ov_ratio_R(int(g0.shape[0]), int(ge.shape[0]), ge.ctypes.data_as(pd), g0.ctypes.data_as(pd),
                        out.ctypes.data_as(pd))
    return rc, out


def test_ratio_matches_oracle():
    rng = np.random.default_rng(3)
    ge = rng.uniform(0.5, 2.0, (4, 48)) * np.exp(-0.3 * np.arange(48))
    g0 = rng.uniform(0.5, 2.0, 48) * np.exp(-0.3 * np.arange(48))
    rc, R = _call(ge, g0)
    assert rc == 0
    ref = corr.ratio(ge.mean(axis=0), g0)
    assert np.abs(R - ref).max() <= 1e-15 * np.abs(ref).max()
    # one field correlator: the plain quotient
    rc, R1 = _call(ge[:1], g0)
    assert rc == 0 and np.array_equal(R1, ge[0] / g0)


def test_ratio_rejects_invalid_correlators():
    g0 = np.ones(8)
    ge = np.ones((4, 8))
    bad = g0.copy()
    bad[3] = 0.0
    assert _call(ge, bad)[0] == -1                  # OV_EINVAL: G_0 must be positive
    bad[3] = np.nan
    assert _call(ge, bad)[0] == -1
    ge2 = ge.copy()
    ge2[1, 5] = np.inf
    assert _call(ge2, g0)[0] == -5                  # OV_ENAN
    lib = ctypes.CDLL(LIB)
    assert lib.ov_ratio_R(0, 1, None, None, None) == -1
