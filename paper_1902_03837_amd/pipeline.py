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


def chi0_pref(cr) -> float:
    """Prefactor of Eq. (X_IP) passed to xo_chi0: f_s / (N_k Omega), f_s = 2 (spin-unpolarised),
    Omega the primitive-cell volume |det(a1, a2, a3)|."""
    return 2.0 / (len(cr.kf) * abs(float(np.linalg.det(cr.lat.avec))))


def nk_omega(cr) -> float:
    """N_k Omega (bohr^3) of the crystal's k-grid, passed to the self-energy calls."""
    return len(cr.kf) * abs(float(np.linalg.det(cr.lat.avec)))


def qpg(cr) -> np.ndarray:
    """|q+G| (1/bohr) over the G-set for xo_epsinv; at q = 0 the G = 0 entry is 1, the head and
    wings of chi0 being the q-normalised limits there."""
    g = (np.asarray(cr.qf, float)[None, :] + cr.gmill.astype(np.float64)) @ cr.lat.bvec
    n = np.sqrt(np.einsum("ij,ij->i", g, g))
    n[n < 1e-12] = 1.0
    return n


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
    xo.chi0(M, dE, cr.omegas, chi0_pref(cr), out=chi, prec=chi_prec or dc.prec, check_dE=check_dE, stream=stream)
    xo.epsinv(chi, qpg(cr), out=E, stream=stream)
    return M, dE, chi, E


class SigmaPlan:
    """Device buffers and per-q argument lists for the self-energy of states at one k-point."""

    def __init__(self, dc: DeviceCrystal, crs, ik0: int, states: slice):
        assert dc.prec == "fp64", "the self-energy path takes FP64 orbitals"
        self.dc, self.crs, self.ik0, self.states = dc, crs, ik0, states
        dev = dc.coef[0].device
        self.nn = states.stop - states.start
        self.rho_plan = None
        self.qs = []
        for cr in crs:
            ik, ikp, g0 = cr.pairs[ik0]
            assert ik == ik0 and np.all(cr.gmill[0] == 0)
            ng, nb = cr.gmill.shape[0], dc.coef[ikp].shape[0]
            f = torch.zeros(nb, dtype=torch.float64, device=dev)
            f[:cr.nocc_at(ikp)] = 1.0
            self.qs.append(dict(ikp=ikp, g0=g0, ng=ng, nb=nb, qpg=qpg(cr), q0=cr.q0, nko=nk_omega(cr), f=f, cr=cr,
                                rho=torch.empty((self.nn, nb, ng), dtype=torch.complex128, device=dev),
                                wr=torch.empty((ng, ng), dtype=torch.complex128, device=dev),
                                om=torch.empty((ng, ng), dtype=torch.complex128, device=dev)))


def sigma_kpoint(plan: SigmaPlan, einv_by_q, z, sigc, sigx, eta=0.0, omega_p=1.0, stream=None):
    """Sigma_x and Sigma_c of the planned states, summed over q: the oscillator strengths
    of every q in one xo_rho_batch (in their mirrored form, every band at k - q on the
    conduction side against the states at k; no q -> 0 substitution), then per q one
    xo_ppa_fit on eps~^-1 at (0, i omega_p) and one xo_sigma."""
    dc, st = plan.dc, plan.states
    if plan.rho_plan is None:
        calls = []
        for Q in plan.qs:
            cr, ikp = Q["cr"], Q["ikp"]
            # mirrored strengths <m k-q| e^{i(-q-G).r} |n k> = conj(rho_nm(q, G)): the bands on
            # the conduction side, the states on the valence side, G0 and the G-set negated
            calls.append(dict(coef_c=dc.coef[ikp], mill_c=cr.mill[ikp], e_c=None,
                              coef_v=dc.coef[plan.ik0][st], mill_v=cr.mill[plan.ik0], e_v=None,
                              gmill=-np.asarray(cr.gmill), g0=-np.asarray(Q["g0"]), grid=cr.grid, out=Q["rho"],
                              prec="fp64", kcart=cr.kcart(ikp), bvec=cr.lat.bvec))
        plan.rho_plan = xo.RhoPlan(calls, batch=True)
    xo.launch_plan(plan.rho_plan, stream=stream)
    for iq, Q in enumerate(plan.qs):
        cr, ikp = Q["cr"], Q["ikp"]
        E = einv_by_q[iq]
        xo.ppa_fit(E[0], E[1], omega_p, Q["qpg"], q0=Q["q0"], nk_omega=Q["nko"], wr=Q["wr"], om=Q["om"],
                   stream=stream)
        xo.sigma(Q["rho"], Q["wr"], Q["om"], dc.eps[ikp], Q["f"], z, eta, Q["nko"], sigc=sigc, sigx=sigx,
                 qpg=Q["qpg"], q0=Q["q0"], accumulate=iq > 0, swapped=True, stream=stream)
    return sigc, sigx


def run_crystal_real(dc: DeviceCrystal, omegas, eta: float, nempty=None, chi_prec=None, M=None, dE=None,
                     chi=None, E=None, check_dE=True, stream=None):
    """The path at real frequencies w + i eta: rho for all pairs, xo_chi0_real and
    xo_epsinv with the LU fallback (eps~ is not Hermitian there); returns (M, dE, chi0, eps~^-1)."""
    cr = dc.cr
    ng, nw = cr.gmill.shape[0], len(omegas)
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
    xo.chi0_real(M, dE, omegas, eta, chi0_pref(cr), out=chi, prec=chi_prec or dc.prec, check_dE=check_dE,
                 stream=stream)
    xo.epsinv(chi, qpg(cr), out=E, flags=xo.XO_EPS_SYM | xo.XO_EPS_LU_FALLBACK, stream=stream)
    return M, dE, chi, E
