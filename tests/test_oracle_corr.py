"""Pins of the correlator oracle (CPU): brute force, a point delta, and the time-reflection
symmetry of the free pion correlator built from dense overlap propagators."""
import numpy as np

import synth
from oracle import api, corr, dense

MW = -1.5


def test_slice_norm2_brute_force():
    L = (2, 3, 2, 4)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, synth.volume(L), 4, 3)) + 1j * rng.standard_normal((3, synth.volume(L), 4, 3))
    ref = np.zeros((3, L[3]))
    C = synth.coords(L)
    for j in range(3):
        for i in range(synth.volume(L)):
            ref[j, C[i, 3]] += sum(abs(x[j, i, s, c]) ** 2 for s in range(4) for c in range(3))
    assert np.abs(corr.slice_norm2(x, L) - ref).max() < 1e-12


def test_point_delta():
    L = (2, 2, 2, 5)
    x = np.zeros((1, synth.volume(L), 4, 3), complex)
    x[0, synth.site_index(L, 1, 0, 1, 3), 2, 1] = 2.0
    g = corr.slice_norm2(x, L)[0]
    assert g[3] == 4.0 and np.count_nonzero(g) == 1


def test_free_pion_correlator_is_time_symmetric():
    """Free field, antiperiodic time: G(t) = G(Lt - t) for a source at t = 0; and it decays
    away from the source."""
    L, bc = (2, 2, 2, 8), (0, 0, 0, 1)
    U = synth.su3_links(L, 0.0, 0)
    H = dense.dense_hw(L, bc, MW, U)
    S = dense.exact_sign(H)
    D = dense.dense_dm(S, 0.2)
    b = synth.point_sources(L, (0, 0, 0, 0))
    props = np.stack([np.linalg.solve(D, bj.ravel()).reshape(bj.shape) for bj in b])
    G = corr.pion_correlator(props, L)
    for t in range(1, L[3]):
        assert abs(G[t] - G[L[3] - t]) < 1e-10 * G[0]
    assert G[0] > G[1] > G[2] > G[3] > G[4]
