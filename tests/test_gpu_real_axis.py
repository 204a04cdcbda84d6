"""GPU parity of the real-axis response (xo_chi0_real) and its Dyson step.

Random transition sets in every precision against the FP64 oracle (frequencies at
zero, between and on the poles; several frequency chunks; accumulate), then the
whole chain for the c1 crystal family at real frequencies: rho, chi0(w + i eta),
eps~^-1 by xo_epsinv with XO_EPS_LU_FALLBACK, against the oracle's chain, and the
reduced forms against FP64.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from synth import crystal_for  # noqa: E402
from synth.rand import random_complex, random_positive  # noqa: E402
from oracle.chi0 import chi0_real_axis, pole_factor_real_axis, crystal_prefactor  # noqa: E402
from oracle.epsinv import epsinv_sym, crystal_qpg  # noqa: E402
from oracle.pipeline import rho_all_pairs  # noqa: E402
from paper_1902_03837_amd import xo  # noqa: E402
from paper_1902_03837_amd.pipeline import DeviceCrystal, run_crystal_real  # noqa: E402

DEV = "cuda"
BF16_U = 2.0 ** -8
TOLS = {"fp64": 1e-13, "fp32": 2e-5, "bf16x3": 2e-4}


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    xo.lib()


def _bf16_bound(M, dE, ws, eta, pref):
    """Plain bf16: each of the Hermitian parts A (weights Re F) and B (Im F) obeys the
    elementwise bound of the imaginary-axis update with |W| for W; the error of A + i B
    is at most the sum."""
    aM = np.abs(M)
    c = np.sqrt(2.0) * (2 * BF16_U + BF16_U ** 2 + M.shape[0] * 2.0 ** -24) * (1 + 2.0 ** -22) * pref
    out = []
    for w in ws:
        F = pole_factor_real_axis(dE, w, eta)
        out.append(c * ((aM.T * (np.abs(F.real) + np.abs(F.imag))) @ aM))
    return np.array(out)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16"])
def test_chi0_real_matches_oracle(prec):
    nt, ng = 700, 97
    M = random_complex(31, (nt, ng), 0.3)
    dE = random_positive(32, nt, 0.1, 2.0)
    ws = [0.0, 0.05, 0.4, float(dE[3]), 1.3, 2.5]   # one frequency exactly on a pole
    eta, pref = 0.02, 0.017
    say(f"chi0_real {prec} nt={nt} ng={ng} nw={len(ws)}")
    ref = chi0_real_axis(M, dE, ws, eta, pref)
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    out = torch.empty((len(ws), ng, ng), dtype=torch.complex128, device=DEV)
    xo.chi0_real(torch.from_numpy(M).to(DEV, cdt), torch.from_numpy(dE).to(DEV), ws, eta, pref, out=out, prec=prec)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    if prec == "bf16":
        Mr = M.astype(np.complex64).astype(np.complex128)   # the device holds complex64 rho
        err = np.abs(got - chi0_real_axis(Mr, dE, ws, eta, pref))
        bound = _bf16_bound(Mr, dE, ws, eta, pref)
        say(f"  max err / bound {np.max(err / bound):.3f}")
        assert np.all(err <= bound)
    else:
        rel = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        say(f"  max rel err {rel:.2e}")
        assert rel <= TOLS[prec]


def test_chi0_real_chunks_and_accumulate():
    nt, ng = 200, 70
    M = random_complex(41, (nt, ng), 0.3)
    dE = random_positive(42, nt, 0.1, 2.0)
    ws = list(np.linspace(0.0, 3.0, 70))   # three chunks of at most 32
    eta, pref = 0.05, 0.02
    ref = chi0_real_axis(M, dE, ws, eta, pref)
    out = torch.full((len(ws), ng, ng), 1.0 + 1.0j, dtype=torch.complex128, device=DEV)
    args = (torch.from_numpy(M).to(DEV), torch.from_numpy(dE).to(DEV), ws, eta, pref)
    xo.chi0_real(*args, out=out)
    torch.cuda.synchronize()
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(ref))
    xo.chi0_real(*args, out=out, accumulate=True)
    torch.cuda.synchronize()
    assert np.max(np.abs(out.cpu().numpy() - 2 * ref)) <= 2e-13 * np.max(np.abs(ref))


def test_chi0_real_rejects_bad_pole_energies():
    M = torch.ones((4, 3), dtype=torch.complex128, device=DEV)
    dE = torch.tensor([0.5, -0.1, 0.3, 0.2], dtype=torch.float64, device=DEV)
    out = torch.empty((1, 3, 3), dtype=torch.complex128, device=DEV)
    with pytest.raises(xo.XoError):
        xo.chi0_real(M, dE, [0.5], 0.01, 1.0, out=out)


def test_real_axis_chain_c1_small():
    """c1 family (fcc, 4 k, 8 occupied + 12 empty bands, NG = 59): eps~^-1(w + i eta) at
    frequencies across the transition range, FP64 against the oracle's chain, the reduced
    forms against FP64."""
    cr = crystal_for("c1_small")
    ws = [0.0, 0.2, 0.45, 0.7, 1.0]
    eta = 0.0037   # 0.1 eV
    say("real-axis chain: oracle")
    M, dE = rho_all_pairs(cr)
    chi_ref = chi0_real_axis(M, dE, ws, eta, crystal_prefactor(cr))
    E_ref = epsinv_sym(chi_ref, crystal_qpg(cr), check=False)
    Es = {}
    for prec in ["fp64", "bf16x3", "bf16"]:
        say(f"real-axis chain: {prec}")
        dc = DeviceCrystal.upload(cr, prec)
        _, _, chi, E = run_crystal_real(dc, ws, eta)
        torch.cuda.synchronize()
        Es[prec] = E.cpu().numpy()
        if prec == "fp64":
            rc = np.max(np.abs(chi.cpu().numpy() - chi_ref)) / np.max(np.abs(chi_ref))
            re = max(np.linalg.norm(Es[prec][j] - E_ref[j]) / np.linalg.norm(E_ref[j]) for j in range(len(ws)))
            say(f"  chi0 rel err {rc:.2e}, eps~^-1 e_F {re:.2e}")
            assert rc < 1e-11 and re < 1e-10
        else:
            eF = max(np.linalg.norm(Es[prec][j] - Es["fp64"][j]) / np.linalg.norm(Es["fp64"][j]) for j in range(len(ws)))
            say(f"  e_F vs fp64 {eF:.2e}")
            # split bf16 against the 1e-4 target; plain bf16 (not a split form, no correction)
            # against its measured error near the poles on this small chain, about 1.5e-3
            assert eF < (1e-4 if prec == "bf16x3" else 2e-3)
