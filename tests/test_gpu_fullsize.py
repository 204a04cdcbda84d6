"""The benchmark workloads at full size, in the launch configuration bench.py times: c2 (64
k-pairs, 16 + 200 bands, 36^3, NG = 400, 8 frequencies, K = 204 800) with sampled columns of
rho and of chi0 against the oracle computed column by column and properties of eps~^-1 that
hold at any size; the large cell at its real G-set and grid with fewer bands; and chi0 at the
large cell's full shape (K = 2 048 000, NG = 3000, 16 frequencies) on sampled elements."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth import crystal_for  # noqa: E402
from oracle.rho import rho_direct  # noqa: E402
from oracle.chi0 import chi0_from_rho, crystal_prefactor  # noqa: E402
from oracle.epsinv import eps_tilde, crystal_qpg  # noqa: E402
from paper_1902_03837_amd import xo  # noqa: E402
from paper_1902_03837_amd.pipeline import DeviceCrystal, run_crystal  # noqa: E402

SAMPLE = [0, 1, 7, 58, 211, 399]


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def c2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    xo.lib()
    cr = crystal_for("c2")
    # oracle: the sampled G columns of rho for every pair, by the direct plane-wave sum
    Ms, dEs = [], []
    for ik, ikp, g0 in cr.pairs:
        cc, cv = cr.coef[ik][cr.nocc:], cr.coef[ikp][:cr.nocc]
        r = rho_direct(cc, cr.mill[ik], cv, cr.mill[ikp], cr.gmill[SAMPLE], g0)
        Ms.append(r.reshape(-1, len(SAMPLE)))
        dEs.append((cr.eps[ik][cr.nocc:][None, :] - cr.eps[ikp][:cr.nocc][:, None]).reshape(-1))
    Mref, dEref = np.concatenate(Ms), np.concatenate(dEs)
    chiref = chi0_from_rho(Mref, dEref, cr.omegas, crystal_prefactor(cr))
    return cr, Mref, dEref, chiref, {}


# Plain bf16 (unit roundoff U = 2^-8 per operand, FP32 accumulation): with normalised
# orbitals each rho is off by at most 2U + U^2 + npw 2^-24 (absolute); chi0 then by at
# most sum_t W_t [(|rho| + d)(|rho'| + d)(1 + sqrt(2) (2U + U^2 + kper 2^-24)) - |rho| |rho'|]
# times pref, elementwise, d being that rho bound and kper <= 65536 the transitions one
# FP32 accumulator sums.
U = 2.0 ** -8


@pytest.mark.parametrize("prec,rtol_rho,rtol_chi", [("fp64", 1e-12, 1e-12), ("bf16x3", 5e-5, 5e-5),
                                                    ("bf16", None, None)])
def test_c2_full_size_sampled(c2, prec, rtol_rho, rtol_chi):
    cr, Mref, dEref, chiref, keep = c2
    say(f"c2 full size {prec}")
    dc = DeviceCrystal.upload(cr, prec)
    M, dE, chi, E = run_crystal(dc, check_dE=False)
    torch.cuda.synchronize()
    Mg = M[:, SAMPLE].cpu().numpy().astype(np.complex128)
    erho = np.abs(Mg - Mref).max() / np.abs(Mref).max()
    chig = chi.cpu().numpy()[:, SAMPLE][:, :, SAMPLE]
    echi = np.abs(chig - chiref).max() / np.abs(chiref).max()
    say(f"  sampled rho err {erho:.2e}, sampled chi0 err {echi:.2e}")
    if rtol_rho is None:
        d = 2 * U + U * U + max(len(m) for m in cr.mill) * 2.0 ** -24
        assert np.abs(Mg - Mref).max() <= d
        a = np.abs(Mref)
        f = 1 + np.sqrt(2.0) * (2 * U + U * U + 65536 * 2.0 ** -24)
        hi = np.abs(chi0_from_rho((a + d).astype(np.complex128), dEref, cr.omegas, crystal_prefactor(cr)))
        lo = np.abs(chi0_from_rho(a.astype(np.complex128), dEref, cr.omegas, crystal_prefactor(cr)))
        ratio = (np.abs(chig - chiref) / (f * hi - lo)).max()
        say(f"  sampled chi0 err / elementwise bound {ratio:.2e}")
        assert ratio <= 1.0
    else:
        assert erho < rtol_rho and echi < rtol_chi
    # eps~^-1 at full size: inverse of the eps~ built from the returned chi0, Hermitian, spectrum in (0, 1]
    chi_h, E_h = chi.cpu().numpy(), E.cpu().numpy()
    et = eps_tilde(chi_h, crystal_qpg(cr))
    for j in range(len(cr.omegas)):
        assert np.abs(et[j] @ E_h[j] - np.eye(et.shape[-1])).max() < 1e-10
        assert np.abs(E_h[j] - E_h[j].conj().T).max() < 1e-10
        ev = np.linalg.eigvalsh(0.5 * (E_h[j] + E_h[j].conj().T))
        assert ev.min() > 0 and ev.max() <= 1 + 1e-10
    # the reduced forms against the plain FP64 path on the whole eps~^-1: the 1e-4 gate
    keep[prec] = E_h
    if prec != "fp64" and "fp64" in keep:
        E64 = keep["fp64"]
        e_f = max(np.linalg.norm(E_h[j] - E64[j]) / np.linalg.norm(E64[j]) for j in range(len(cr.omegas)))
        say(f"  eps~^-1 {prec} vs fp64: {e_f:.2e}")
        assert e_f < 1e-4


# ------------------------------------------------------------------ large cell
C5S = [0, 1, 17, 500, 1999, 2999]


@pytest.fixture(scope="module")
def c5s():
    """The large cell at its real G-set (NG = 3000) and 72^3 grid, k = {Gamma, b1/2},
    128 occupied + 200 empty bands, 4 frequencies: K = 51 200."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    xo.lib()
    cr = crystal_for("c5_small")
    Ms, dEs = [], []
    for ik, ikp, g0 in cr.pairs:
        cc, cv = cr.coef[ik][cr.nocc:], cr.coef[ikp][:cr.nocc]
        Ms.append(rho_direct(cc, cr.mill[ik], cv, cr.mill[ikp], cr.gmill[C5S], g0).reshape(-1, len(C5S)))
        dEs.append((cr.eps[ik][cr.nocc:][None, :] - cr.eps[ikp][:cr.nocc][:, None]).reshape(-1))
    Mref, dEref = np.concatenate(Ms), np.concatenate(dEs)
    return cr, Mref, dEref, chi0_from_rho(Mref, dEref, cr.omegas, crystal_prefactor(cr)), {}


def check_plain_bf16(cr, Mg, Mref, dEref, chig, chiref):
    """Plain bf16 against its rounding bounds (see the c2 test): rho absolutely, chi0 element-wise."""
    d = 2 * U + U * U + max(len(m) for m in cr.mill) * 2.0 ** -24
    assert np.abs(Mg - Mref).max() <= d
    a = np.abs(Mref)
    f = 1 + np.sqrt(2.0) * (2 * U + U * U + 65536 * 2.0 ** -24)
    hi = np.abs(chi0_from_rho((a + d).astype(np.complex128), dEref, cr.omegas, crystal_prefactor(cr)))
    lo = np.abs(chi0_from_rho(a.astype(np.complex128), dEref, cr.omegas, crystal_prefactor(cr)))
    ratio = (np.abs(chig - chiref) / (f * hi - lo)).max()
    say(f"  sampled chi0 err / elementwise bound {ratio:.2e}")
    assert ratio <= 1.0


@pytest.mark.parametrize("prec,rtol_rho,rtol_chi", [("fp64", 1e-12, 1e-12), ("bf16x3", 5e-5, 5e-5),
                                                    ("bf16", None, None)])
def test_c5_small_real_gset(c5s, prec, rtol_rho, rtol_chi):
    cr, Mref, dEref, chiref, keep = c5s
    say(f"large cell, NG = 3000, {prec}")
    dc = DeviceCrystal.upload(cr, prec)
    M, dE, chi, E = run_crystal(dc, check_dE=False)
    torch.cuda.synchronize()
    Mg = M[:, C5S].cpu().numpy().astype(np.complex128)
    erho = np.abs(Mg - Mref).max() / np.abs(Mref).max()
    chig = chi[:, C5S][:, :, C5S].cpu().numpy()
    echi = np.abs(chig - chiref).max() / np.abs(chiref).max()
    say(f"  sampled rho err {erho:.2e}, sampled chi0 err {echi:.2e}")
    if rtol_rho is None:
        check_plain_bf16(cr, Mg, Mref, dEref, chig, chiref)
    else:
        assert erho < rtol_rho and echi < rtol_chi
    keep[prec] = (chi.cpu().numpy() if prec == "fp64" else None, E.cpu().numpy())
    if prec == "fp64":
        # FP64 eps~^-1 of one frequency against the oracle's inverse of the same chi0
        from oracle.epsinv import epsinv_sym
        c64, E64 = keep["fp64"]
        ref = epsinv_sym(c64[1:2], crystal_qpg(cr))
        assert np.abs(E64[1] - ref[0]).max() < 1e-10 * np.abs(ref[0]).max()
    elif "fp64" in keep:
        # reduced precision against the plain FP64 path on the whole eps~^-1
        E64, Er = keep["fp64"][1], keep[prec][1]
        e_f = max(np.linalg.norm(Er[j] - E64[j]) / np.linalg.norm(E64[j]) for j in range(len(cr.omegas)))
        say(f"  eps~^-1 {prec} vs fp64: {e_f:.2e}")
        assert e_f < 1e-4


# --------------------------------------------------------------------------------------
# Every form's eps~^-1 at full size against the oracle's (c2: all 64 k-pairs, 204 800
# transitions, NG = 400, 8 frequencies; the oracle's FFT route, zgemm and LU on the host
# cores, about half a minute). The chosen forms (FP32, split bf16) are held to the 1e-4 target
# of the relative Frobenius error at every frequency, plain FP64 to 1e-6 (it reaches ~1e-14).
# Plain bf16 is not a chosen form (no split correction; its element-wise rounding bounds are
# asserted above): its error here is reported and held to the bound measured for this
# workload, 5e-5.

@pytest.fixture(scope="module")
def c2_oracle_eps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    xo.lib()
    from oracle.pipeline import epsinv_crystal
    cr = crystal_for("c2")
    say("oracle eps~^-1 of c2 at full size (host cores)")
    E, _ = epsinv_crystal(cr)
    return cr, E


@pytest.mark.parametrize("prec,gate", [("fp64", 1e-6), ("fp32", 1e-4), ("bf16x3", 1e-4), ("bf16", 5e-5)])
def test_c2_eps_every_form_vs_oracle(c2_oracle_eps, prec, gate):
    cr, Eref = c2_oracle_eps
    dc = DeviceCrystal.upload(cr, prec)
    _, _, _, E = run_crystal(dc, check_dE=False)
    torch.cuda.synchronize()
    Eg = E.cpu().numpy()
    e_f = max(np.linalg.norm(Eg[j] - Eref[j]) / np.linalg.norm(Eref[j]) for j in range(len(cr.omegas)))
    say(f"  c2 full size {prec}: e_F(eps~^-1) vs oracle {e_f:.2e}")
    assert e_f <= gate
    if prec == "fp64":
        assert e_f < 1e-11


# --------------------------------------------------------------------------------------
# chi0 at the full large-cell shape (K = 2 048 000 transitions, NG = 3000, the 16 imaginary
# frequencies of the workload), through the same call and automatic unit slicing bench.py
# times. The strengths are seeded random numbers drawn on the device (49 GB in complex64);
# the oracle sums all 2 048 000 transitions for the sampled (G, G') pairs, which span the
# first and last 64-blocks, the diagonal and the ragged edge of the G-set. Tolerances as in
# the random chi0 tests: FP64 1e-12, FP32 2e-5 and split bf16 2e-4 of the largest sampled
# element. The whole result is exactly Hermitian.

@pytest.mark.parametrize("prec,tol", [("bf16x3", 2e-4), ("fp32", 2e-5), ("fp64", 1e-12)])
def test_chi0_full_large_cell_shape_sampled(prec, tol):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from synth.rand import device_random_rho
    from synth.crystal import frequencies
    xo.lib()
    K, NG = 2_048_000, 3000
    w = frequencies(16)
    dev = torch.device("cuda:0")
    say(f"chi0 at the full large-cell shape, {prec}: K={K}, NG={NG}, 16 frequencies")
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    M, dE = device_random_rho(11, K, NG, dt, dev)
    out = torch.empty((len(w), NG, NG), dtype=torch.complex128, device=dev)
    xo.chi0(M, dE, w, 1.0, out=out, prec=prec, check_dE=False)
    torch.cuda.synchronize()
    herm = bool(torch.equal(out, out.conj().transpose(1, 2)))
    Ms = M[:, C5S].cpu().numpy().astype(np.complex128)
    dEs = dE.cpu().numpy()
    got = out[:, C5S][:, :, C5S].cpu().numpy()
    del M, dE, out
    torch.cuda.empty_cache()
    ref = chi0_from_rho(Ms, dEs, w, 1.0)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  sampled chi0 err {err:.2e} (tolerance {tol:.0e}), exactly Hermitian: {herm}")
    assert herm
    assert err < tol
