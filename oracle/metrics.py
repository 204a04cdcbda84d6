"""Error measures used to gate results against the oracle. TEST INFRASTRUCTURE (oracle).

e_F = max over frequencies of ||E - E_ref||_F / ||E_ref||_F for E = eps~^-1;
e_S = the same error over ||E_ref - I||_F (the screening part only);
head = |E_00 - E_ref,00| / |E_ref,00|; chi0 error = relative Frobenius error.
"""

from __future__ import annotations

import numpy as np


def rel_fro(a, b) -> float:
    """max over the leading axis of ||a - b||_F / ||b||_F (2-D inputs: one value)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.ndim == 2:
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return max(float(np.linalg.norm(a[i] - b[i]) / np.linalg.norm(b[i])) for i in range(a.shape[0]))


def err_table(E, Eref, chi=None, chiref=None) -> dict:
    E = np.asarray(E)
    Eref = np.asarray(Eref)
    ng = E.shape[-1]
    eye = np.eye(ng)
    eF = rel_fro(E, Eref)
    eS = max(float(np.linalg.norm(E[i] - Eref[i]) / np.linalg.norm(Eref[i] - eye))
             for i in range(E.shape[0]))
    head = max(float(abs(E[i, 0, 0] - Eref[i, 0, 0]) / abs(Eref[i, 0, 0])) for i in range(E.shape[0]))
    out = dict(e_F=eF, e_S=eS, head=head)
    if chi is not None:
        out["chi0"] = rel_fro(chi, chiref)
    return out
