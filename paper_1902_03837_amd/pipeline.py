"""Drive a whole crystal through libxo: every k-pair -> rho -> chi0 -> eps~^-1.

Host work here is argument marshalling only (slicing device tensors, passing
the host Miller lists); every arithmetic step runs in the HIP kernels.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import xo

CDTYPE = {"fp64": torch.complex128, "fp32": torch.complex64, "bf16x3": torch.complex64, "bf16": torch.complex64}


@dataclass
class DeviceCrystal:
    """Orbitals and energies of a crystal resident in device memory."""
    cr: object
    prec: str
    coef: List[torch.Tensor]
    eps: List[torch.Tensor]
    plans: dict = None

    def __post_init__(self):
        if self.plans is None:
            self.plans = {}

    @classmethod
    def upload(cls, cr, prec="fp64", device="cuda"):
        cdt = CDTYPE[prec]
        coef = [torch.from_numpy(np.ascontiguousarray(c)).to(device=device, dtype=cdt) for c in cr.coef]
        eps = [torch.from_numpy(np.ascontiguousarray(e)).to(device=device, dtype=torch.float64) for e in cr.eps]
        return cls(cr, prec, coef, eps)


def band_ranges(cr, nempty: Optional[int] = None, band_lo: Optional[int] = None):
    """Per pair: (ik, ik', g0, conduction slice, valence count) in transition order."""
    out = []
    for ik, ikp, g0 in cr.pairs:
        lo = cr.nocc_at(ik) if band_lo is None else band_lo
        hi = cr.coef[ik].shape[0] if nempty is None else cr.nocc_at(ik) + nempty
        out.append((ik, ikp, g0, lo, hi, cr.nocc_at(ikp)))
    return out


def ntrans(cr, nempty=None, band_lo=None) -> int:
    return sum((hi - lo) * nv for _, _, _, lo, hi, nv in band_ranges(cr, nempty, band_lo))


def rho_all(dc: DeviceCrystal, M: torch.Tensor, dE: torch.Tensor, nempty=None, band_lo=None,
            qhat=(1.0, 0.0, 0.0), rho_prec=None, stream=None, batch=True):
    """Fill M[K][ng] and dE[K] for every pair (transition t = v * nc + c within a pair).

    batch=True passes every pair to one xo_rho_batch call; batch=False calls xo_rho per pair.
    """
    cr = dc.cr
    ng = cr.gmill.shape[0]
    key = (M.data_ptr(), dE.data_ptr(), nempty, band_lo, tuple(qhat), rho_prec, batch)
    plan = dc.plans.get(key)
    if plan is not None:
        xo.launch_plan(plan, stream=stream)
        return plan.ntrans
    off = 0
    calls = []
    for ik, ikp, g0, lo, hi, nv in band_ranges(cr, nempty, band_lo):
        nc = hi - lo
        n = nc * nv
        calls.append(dict(coef_c=dc.coef[ik][lo:hi], mill_c=cr.mill[ik], e_c=dc.eps[ik][lo:hi],
                          coef_v=dc.coef[ikp][:nv], mill_v=cr.mill[ikp], e_v=dc.eps[ikp][:nv],
                          gmill=cr.gmill, g0=g0, grid=cr.grid, out=M[off:off + n].view(nv, nc, ng),
                          dE=dE[off:off + n], prec=rho_prec or dc.prec, kcart=cr.kcart(ik), bvec=cr.lat.bvec,
                          q0=cr.q0, qhat=qhat))
        off += n
    plan = xo.RhoPlan(calls, batch, off)
    dc.plans[key] = plan
    xo.launch_plan(plan, stream=stream)
    return off


def run_crystal(dc: DeviceCrystal, nempty=None, chi_prec=None, M=None, dE=None, chi=None, E=None,
                check_dE=True, stream=None):
    """Whole path for one crystal; returns (M, dE, chi0, eps~^-1) device tensors."""
    cr = dc.cr
    ng, nw = cr.gmill.shape[0], len(cr.omegas)
    K = ntrans(cr, nempty)
    dev = dc.coef[0].device
    if M is None:
        M = torch.empty((K, ng), dtype=CDTYPE[dc.prec], device=dev)
    if dE is None:
        dE = torch.empty(K, dtype=torch.float64, device=dev)
    if chi is None:
        chi = torch.empty((nw, ng, ng), dtype=torch.complex128, device=dev)
    if E is None:
        E = torch.empty_like(chi)
    rho_all(dc, M, dE, nempty, stream=stream)
    xo.chi0(M, dE, cr.omegas, cr.pref, out=chi, prec=chi_prec or dc.prec, check_dE=check_dE, stream=stream)
    xo.epsinv(chi, cr.qpg(), out=E, stream=stream)
    return M, dE, chi, E
