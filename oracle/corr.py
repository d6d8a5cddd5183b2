"""Pion correlators and the ratio R(t) (TEST INFRASTRUCTURE ONLY).

Sec. 4: the energy shift of the neutral pion in an electric field comes from
R(t) = G_E(t) / G_0(t), G_E from propagators in the field (u and d quarks,
both signs of the field), G_0 without it.  With gamma5-hermiticity of D(m),
the connected pseudoscalar correlator of one flavour from point-source
propagators S_j (source spin-colour j, sink site x) is
    G(t) = sum_{x in time slice t} sum_j sum_{s, c} |S_j(x)_{s c}|^2.
Written out here from that definition, independently of the library.
"""
from __future__ import annotations

import numpy as np


def slice_norm2(x, L):
    """(n, Lt): sum over each time slice and the 12 components of |x_j|^2; x (n, V, 4, 3)."""
    x = np.asarray(x)
    Lx, Ly, Lz, Lt = L
    n = x.shape[0]
    a = np.abs(x.reshape(n, Lt, Lz * Ly * Lx * 12)) ** 2   # canonical order: t slowest
    return a.sum(axis=2)


def pion_correlator(props, L):
    """G(t) of one flavour from its 12 point-source propagators (12, V, 4, 3)."""
    return slice_norm2(props, L).sum(axis=0)


def ratio(G_E, G_0):
    return np.asarray(G_E) / np.asarray(G_0)
