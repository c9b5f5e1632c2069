"""Conjugate symmetry of the frequency set (oracle).

The kernel satisfies U(r, conj(s)) = conj(U(r, s)), so V(conj s) = conj(V(s))
entry by entry; the paper uses this to compute only half of the frequencies
(Sec. 5.1, selected frequencies; App. A, last paragraph).  For a set with
s_{L-k} = conj(s_k) the distinct representatives are k = 0..L/2 and

    V(s_k) x = conj( V(s_{L-k}) conj(x) )   for k > L/2.

``representatives(s)`` returns, for every k, (rep(k), conj flag); with
symmetry disabled every frequency represents itself.
"""
from __future__ import annotations

import numpy as np


def representatives(s, use_symmetry: bool = True, rtol: float = 1e-12):
    s = np.asarray(s, dtype=np.complex128)
    L = len(s)
    rep = np.arange(L)
    conj = np.zeros(L, dtype=bool)
    if use_symmetry:
        for k in range(L // 2 + 1, L):
            j = L - k
            if abs(s[k] - np.conj(s[j])) <= rtol * abs(s[j]):
                rep[k] = j
                conj[k] = True
    return rep, conj


def distinct(rep):
    """Sorted list of the frequencies that represent themselves (the set K)."""
    rep = np.asarray(rep)
    return np.nonzero(rep == np.arange(len(rep)))[0]
