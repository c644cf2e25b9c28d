"""Active-space self-energy correction and Dyson's equation (test infrastructure).

Eqs. 12-14 of the paper, written out with dense inverses:

    Sigma_CAS(k, w)  = G_GW,CAS(k, w)^-1 - G_CC,CAS(k, w)^-1
    Sigma_full(k, w) = V(k) Sigma_CAS(k, w) V(k)^H
    G_CC+GW(k, w)    = [G_GW,full(k, w)^-1 - Sigma_full(k, w)]^-1

Inputs are arrays [..., n, n] (any leading batch axes); V is [..., N, M] with the
active natural orbitals as columns.  Parity: pinned by three closed forms in
tests/test_oracle_dyson.py (an active space where CC equals the low-level
method gives back G_GW; a complete active space gives V G_CC V^H; static
self-energies give the resolvent of the corrected one-body matrix).
"""
from __future__ import annotations

import numpy as np


def sigma_cas(Ggw_cas, Gcc):
    """Eq. 12."""
    return np.linalg.inv(Ggw_cas) - np.linalg.inv(Gcc)


def back_transform(V, S):
    """Eq. 13: V S V^H."""
    return V @ S @ np.conj(np.swapaxes(V, -1, -2))


def dyson(Ggw, Sfull):
    """Eq. 14."""
    return np.linalg.inv(np.linalg.inv(Ggw) - Sfull)


def cc_gw(Ggw, Ggw_cas, Gcc, V):
    """(G_CC+GW, Sigma_full, Sigma_CAS) for Ggw [nk, nw, N, N], Ggw_cas and Gcc
    [nk, nw, M, M], V [nk, N, M]."""
    S = sigma_cas(Ggw_cas, Gcc)
    Sf = back_transform(V[:, None], S)
    return dyson(Ggw, Sf), Sf, S
