"""Parity of the HIP path (through the C-ABI) with the FP64 oracle, element by element."""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth import crystal_for  # noqa: E402
from synth.crystal import fcc_lattice, make_crystal, shell_potential, ecut_for_npw, kgrid_gamma  # noqa: E402
from synth.configs import A_FCC  # noqa: E402
from synth.rand import random_complex, random_positive  # noqa: E402
from oracle.pipeline import rho_pair, rho_all_pairs, chi0_crystal  # noqa: E402
from oracle.chi0 import chi0_from_rho  # noqa: E402
from oracle.epsinv import epsinv_sym, epsinv_nonsym  # noqa: E402
from oracle.metrics import err_table, rel_fro  # noqa: E402
from paper_1902_03837_amd import xo  # noqa: E402
from oracle.epsinv import crystal_qpg  # noqa: E402
from paper_1902_03837_amd.pipeline import DeviceCrystal, run_crystal, rho_all, ntrans  # noqa: E402

DEV = "cuda"


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    xo.lib()


def _to(a, dt=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


# ----------------------------------------------------------------------------- rho

# rho has two kernels in every precision: the gathered product (default where its
# tables fit in LDS) and the transform (axis-factorised on MFMA for the bf16 forms,
# split in both; on VALU for FP32 / FP64); XO_RHO_KERNEL pins one of them.
# tol: max error over max |rho|; None: the plain-bf16 rounding bound below
RHO_FORMS = [("fp64", "gemm", 1e-13), ("fp64", "transform", 1e-13), ("fp32", "gemm", 3e-6),
             ("fp32", "transform", 3e-6), ("bf16x3", "gemm", 5e-5), ("bf16x3", "transform", 5e-5),
             ("bf16", "gemm", None), ("bf16", "transform", 5e-5)]

# Plain bf16 (XO_BF16): every operand rounded to bf16 (unit roundoff U = 2^-8), one
# product per pair, FP32 accumulation (2^-24 per add). A real product of rounded
# operands is off by at most (2U + U^2) |a| |b|, and the real and imaginary parts of a
# complex product each gather at most |a| |b| of such terms (Cauchy-Schwarz), so
#   rho:  |err| <= (2U + U^2 + n 2^-24) sum_a |c_c(a)| |c_v(a - e)| <= 2U + U^2 + n 2^-24
#         for normalised orbitals (n: plane waves summed);
#   chi0: |err_GG'| <= sqrt(2) (2U + U^2 + nt 2^-24) (1 + 2^-22) pref sum_t W_t |rho_t(G)| |rho_t(G')|
#         (the left operand W rho is formed in FP32 before its rounding).
BF16_U = 2.0 ** -8


def bf16_rho_bound(npw):
    return 2 * BF16_U + BF16_U ** 2 + npw * 2.0 ** -24


def bf16_chi0_bound(M, dE, w, pref):
    """Elementwise bound on the plain-bf16 chi0 error, from the oracle's sum of |rho| |rho'|."""
    absum = np.abs(chi0_from_rho(np.abs(M).astype(np.complex128), dE, w, pref))
    return np.sqrt(2.0) * (2 * BF16_U + BF16_U ** 2 + M.shape[0] * 2.0 ** -24) * (1 + 2.0 ** -22) * absum


def check_rho(Mg, Mr, tol, npw):
    if tol is None:
        err = np.abs(Mg - Mr).max()
        say(f"  max abs err {err:.3e} (bound {bf16_rho_bound(npw):.3e}), over max |rho| {err / np.abs(Mr).max():.3e}")
        assert err <= bf16_rho_bound(npw)
    else:
        err = np.abs(Mg - Mr).max() / np.abs(Mr).max()
        say(f"  max rel err {err:.3e}")
        assert err < tol


class rho_kernel:
    """Pin the rho kernel for the calls inside the block and check that it ran."""

    def __init__(self, name, prec="bf16x3"):
        self.name, self.prec = name, prec

    def __enter__(self):
        self.old = os.environ.get("XO_RHO_KERNEL")
        if self.name:
            os.environ["XO_RHO_KERNEL"] = self.name
            xo.timing_enable(True)
        return self

    def __exit__(self, *exc):
        if self.name:
            torch.cuda.synchronize()
            ran = xo.timing_report()
            xo.timing_enable(False)
            if exc[0] is None:
                want = "rho_gemm" if self.name == "gemm" else ("rho_yz" if self.prec.startswith("bf16") else "rho_zy")
                assert any(k.startswith(want) for k in ran), ran.keys()
        if self.old is None:
            os.environ.pop("XO_RHO_KERNEL", None)
        else:
            os.environ["XO_RHO_KERNEL"] = self.old
        return False


@pytest.mark.parametrize("name", ["c1", "c2_small"])
@pytest.mark.parametrize("prec,kern,tol", RHO_FORMS)
def test_rho_parity(name, prec, kern, tol):
    cr = crystal_for(name)
    say(f"rho parity {name} {prec} {kern}")
    dc = DeviceCrystal.upload(cr, prec)
    K = ntrans(cr)
    ng = cr.gmill.shape[0]
    M = torch.empty((K, ng), dtype=torch.complex128 if prec == "fp64" else torch.complex64, device=DEV)
    dE = torch.empty(K, dtype=torch.float64, device=DEV)
    with rho_kernel(kern, prec):
        rho_all(dc, M, dE)
    torch.cuda.synchronize()
    Mr, dEr = rho_all_pairs(cr, "fft")
    Mg = M.cpu().numpy().astype(np.complex128)
    check_rho(Mg, Mr, tol, max(len(m) for m in cr.mill))
    assert np.array_equal(dE.cpu().numpy(), dEr)


@pytest.mark.parametrize("prec,kern,tol", RHO_FORMS)
def test_rho_parity_large_gset(prec, kern, tol):
    """NG = 700 on a 28^3 grid: more G-vectors than one workgroup of the axis-factorised
    kernel owns (the G-set is split into several (e_y, e_z)-column groups); for the
    gathered product, row blocks that straddle two valence bands."""
    cr = crystal_for("c2_small", ng=700, grid=28)
    say(f"rho parity NG=700 {prec} {kern}")
    dc = DeviceCrystal.upload(cr, prec)
    K = ntrans(cr)
    M = torch.empty((K, 700), dtype=torch.complex128 if prec == "fp64" else torch.complex64, device=DEV)
    dE = torch.empty(K, dtype=torch.float64, device=DEV)
    with rho_kernel(kern, prec):
        rho_all(dc, M, dE)
    torch.cuda.synchronize()
    Mr, _ = rho_all_pairs(cr, "fft")
    check_rho(M.cpu().numpy().astype(np.complex128), Mr, tol, max(len(m) for m in cr.mill))


@pytest.mark.parametrize("nempty", [28, 128])
def test_rho_plain_bf16_column_groups(nempty):
    """The plain-bf16 gathered product takes seven column tiles per workgroup when that
    needs no more groups than eight (28 empty bands: 2 tiles), else eight (128: 8 tiles)."""
    cr = crystal_for("c2_small", nempty=nempty)
    say(f"rho plain bf16, {nempty} empty bands")
    dc = DeviceCrystal.upload(cr, "bf16")
    K = ntrans(cr)
    M = torch.empty((K, cr.gmill.shape[0]), dtype=torch.complex64, device=DEV)
    dE = torch.empty(K, dtype=torch.float64, device=DEV)
    with rho_kernel("gemm", "bf16"):
        rho_all(dc, M, dE)
    Mr, _ = rho_all_pairs(cr, "fft")
    check_rho(M.cpu().numpy().astype(np.complex128), Mr, None, max(len(m) for m in cr.mill))


@pytest.mark.parametrize("prec", ["fp64", "bf16x3", "bf16"])
def test_rho_batch_equals_per_pair(prec):
    cr = crystal_for("c2_small")
    say(f"rho batch vs per-pair {prec}")
    dc = DeviceCrystal.upload(cr, prec)
    K = ntrans(cr)
    ng = cr.gmill.shape[0]
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    M1 = torch.empty((K, ng), dtype=cdt, device=DEV)
    M2 = torch.empty_like(M1)
    d1 = torch.empty(K, dtype=torch.float64, device=DEV)
    d2 = torch.empty_like(d1)
    rho_all(dc, M1, d1, batch=True)
    rho_all(dc, M2, d2, batch=False)
    assert torch.equal(M1, M2) and torch.equal(d1, d2)


@pytest.mark.parametrize("prec,kern,tol_head,tol", [("fp64", "gemm", 1e-12, 1e-12), ("fp64", "transform", 1e-12, 1e-12),
                                                    ("bf16x3", "gemm", 1e-6, 5e-5), ("bf16x3", "transform", 1e-6, 5e-5),
                                                    ("bf16", "gemm", 1e-6, None)])
def test_rho_q0_head_parity(prec, kern, tol_head, tol):
    """q -> 0: the G = 0 column is the velocity head (accumulated in FP64 in every
    form, rounded to the output precision); the other columns come from the transform."""
    lat = fcc_lattice(A_FCC)
    cr = make_crystal(lat, shell_potential(lat, 31), kgrid_gamma(2), np.zeros(3), (16,) * 3,
                      ecut_for_npw(lat, 160), 4, 12, 27, 2, 31)
    say(f"rho q0 head parity {prec} {kern}")
    assert cr.q0
    dc = DeviceCrystal.upload(cr, prec)
    K = ntrans(cr)
    M = torch.empty((K, 27), dtype=torch.complex128 if prec == "fp64" else torch.complex64, device=DEV)
    dE = torch.empty(K, dtype=torch.float64, device=DEV)
    with rho_kernel(kern, prec):
        rho_all(dc, M, dE)
    Mr, _ = rho_all_pairs(cr, "fft")
    Mg = M.cpu().numpy().astype(np.complex128)
    assert np.abs(Mg[:, 0] - Mr[:, 0]).max() < tol_head * np.abs(Mr[:, 0]).max()
    if tol is None:
        check_rho(Mg[:, 1:], Mr[:, 1:], None, max(len(m) for m in cr.mill))
    else:
        assert np.abs(Mg - Mr).max() < tol * np.abs(Mr).max()


# ---------------------------------------------------------------------------- chi0

@pytest.mark.parametrize("nt,ng,nw", [(1, 1, 1), (37, 17, 2), (1000, 33, 3), (777, 59, 8), (300, 40, 11)])
def test_chi0_fp64_random(nt, ng, nw):
    say(f"chi0 fp64 random nt={nt} ng={ng} nw={nw}")
    M = random_complex(100 + nt, (nt, ng))
    dE = random_positive(200 + nt, nt, 0.05, 3.0)
    w = np.linspace(0.0, 2.0, nw)
    ref = chi0_from_rho(M, dE, w, 0.37)
    out = torch.empty((nw, ng, ng), dtype=torch.complex128, device=DEV)
    xo.chi0(_to(M), _to(dE, torch.float64), w, 0.37, out=out, prec="fp64")
    got = out.cpu().numpy()
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
    for j in range(nw):
        assert np.array_equal(got[j], got[j].conj().T)   # exactly Hermitian by construction


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-5), ("bf16x3", 2e-4), ("bf16", None)])
@pytest.mark.parametrize("nt,ng,nw", [(5000, 45, 4), (3001, 150, 8), (517, 64, 5)])
def test_chi0_reduced_precision_random(prec, tol, nt, ng, nw):
    say(f"chi0 {prec} random nt={nt} ng={ng} nw={nw}")
    M = random_complex(7, (nt, ng))
    dE = random_positive(8, nt, 0.05, 3.0)
    w = np.linspace(0.0, 2.0, nw)
    ref = chi0_from_rho(M.astype(np.complex64).astype(np.complex128), dE, w, 1.0)
    out = torch.empty((nw, ng, ng), dtype=torch.complex128, device=DEV)
    xo.chi0(_to(M, torch.complex64), _to(dE, torch.float64), w, 1.0, out=out, prec=prec)
    got = out.cpu().numpy()
    err = rel_fro(got, ref)
    say(f"  rel Frobenius err {err:.3e}")
    if tol is None:
        bound = bf16_chi0_bound(M.astype(np.complex64).astype(np.complex128), dE, w, 1.0)
        ratio = (np.abs(got - ref) / bound).max()
        say(f"  max err / elementwise bound {ratio:.3e}")
        assert ratio <= 1.0
    else:
        assert err < tol
    for j in range(nw):
        assert np.array_equal(got[j], got[j].conj().T)
    again = torch.empty_like(out)
    xo.chi0(_to(M, torch.complex64), _to(dE, torch.float64), w, 1.0, out=again, prec=prec)
    assert torch.equal(out, again)   # fixed-order reduction: bitwise repeatable


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("nt,ng,nw,tune", [(1, 1, 1, None), (1, 1, 1, (4, 0, 0)), (33, 17, 1, (4, 0, 0)),
                                           (700, 65, 3, (4, 256, 1)), (130, 129, 6, None),
                                           (1, 1, 1, (8, 0, 0)), (33, 17, 1, (8, 0, 0)), (700, 65, 3, (8, 256, 1)),
                                           (130, 129, 6, (8, 0, 0)), (517, 200, 5, (8, 64, 1)),
                                           (300, 129, 4, (4, 0, 0)), (700, 130, 11, (4, 256, 1)),
                                           (300, 70, 12, None)])
def test_chi0_bf16_edges(prec, nt, ng, nw, tune):
    """Degenerate and ragged shapes of the bf16 forms: one transition, one G-vector, one
    frequency in the 64 x 64 block form (three padded frequency slots) and the 64 x 128
    strip form (one), G-sets one past a block edge, transition slices shorter than a step, three
    frequency groups in the block form (two units in one workgroup, one alone); within the
    bf16 rounding bound (plain) or 2e-4 (split), exactly Hermitian."""
    say(f"chi0 {prec} edge nt={nt} ng={ng} nw={nw} tune={tune}")
    M = random_complex(300 + nt, (nt, ng)).astype(np.complex64).astype(np.complex128)
    dE = random_positive(400 + nt, nt, 0.05, 3.0)
    w = list(np.linspace(0.0, 1.5, nw))
    ref = chi0_from_rho(M, dE, w, 0.8)
    out = torch.empty((nw, ng, ng), dtype=torch.complex128, device=DEV)
    xo.chi0_batch([(_to(M, torch.complex64), _to(dE, torch.float64), 0.8, out)], w, prec=prec, tune=tune)
    got = out.cpu().numpy()
    if prec == "bf16":
        assert (np.abs(got - ref) / bf16_chi0_bound(M, dE, w, 0.8)).max() <= 1.0
    else:
        assert rel_fro(got, ref) < 2e-4
    for j in range(nw):
        assert np.array_equal(got[j], got[j].conj().T)


def test_chi0_bf16_accumulate_chunks():
    """Streaming transitions in chunks (accumulate = 1) adds up to the unsplit result
    within the plain-bf16 bound."""
    nt, ng, nw = 2000, 70, 4
    M = random_complex(21, (nt, ng)).astype(np.complex64).astype(np.complex128)
    dE = random_positive(22, nt, 0.1, 2.0)
    w = [0.0, 0.4, 1.0, 2.0]
    Md, dEd = _to(M, torch.complex64), _to(dE, torch.float64)
    part = torch.empty((nw, ng, ng), dtype=torch.complex128, device=DEV)
    xo.chi0(Md[:700], dEd[:700], w, 1.0, out=part, prec="bf16")
    xo.chi0(Md[700:], dEd[700:], w, 1.0, out=part, prec="bf16", accumulate=True)
    ref = chi0_from_rho(M, dE, w, 1.0)
    assert (np.abs(part.cpu().numpy() - ref) / bf16_chi0_bound(M, dE, w, 1.0)).max() <= 1.0


def test_chi0_accumulate_and_determinism():
    nt, ng, nw = 3000, 50, 3
    M = random_complex(11, (nt, ng))
    dE = random_positive(12, nt, 0.1, 2.0)
    w = [0.0, 0.5, 1.5]
    Md, dEd = _to(M), _to(dE, torch.float64)
    full = torch.empty((nw, ng, ng), dtype=torch.complex128, device=DEV)
    full2 = torch.empty_like(full)
    xo.chi0(Md, dEd, w, 1.0, out=full)
    xo.chi0(Md, dEd, w, 1.0, out=full2)
    assert torch.equal(full, full2)                       # fixed-order reduction
    part = torch.empty_like(full)
    xo.chi0(Md[:1200], dEd[:1200], w, 1.0, out=part)
    xo.chi0(Md[1200:], dEd[1200:], w, 1.0, out=part, accumulate=True)
    a, b = part.cpu().numpy(), full.cpu().numpy()
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()  # sharding invariance


def test_chi0_rejects_nonpositive_pole():
    M = random_complex(1, (10, 4))
    dE = np.ones(10)
    dE[3] = -0.1
    out = torch.empty((1, 4, 4), dtype=torch.complex128, device=DEV)
    with pytest.raises(xo.XoError) as e:
        xo.chi0(_to(M), _to(dE, torch.float64), [0.0], 1.0, out=out)
    assert e.value.code == xo.XO_ERR_ARG


# -------------------------------------------------------------------------- epsinv

@pytest.mark.parametrize("name", ["c1", "c2_small"])
def test_epsinv_parity(name):
    cr = crystal_for(name)
    say(f"epsinv parity {name}")
    chi = chi0_crystal(cr)
    qpg = crystal_qpg(cr)
    ref = epsinv_sym(chi, qpg)
    out = torch.empty(chi.shape, dtype=torch.complex128, device=DEV)
    xo.epsinv(_to(chi), qpg, out=out)
    got = out.cpu().numpy()
    assert rel_fro(got, ref) < 1e-12
    refn = epsinv_nonsym(chi, qpg)
    xo.epsinv(_to(chi), qpg, out=out, flags=xo.XO_EPS_NONSYM)
    assert rel_fro(out.cpu().numpy(), refn) < 1e-12


@pytest.mark.parametrize("rank", ["valu", "mfma"])
@pytest.mark.parametrize("ng", [1, 31, 32, 33, 63, 64, 65, 97, 128, 200])
def test_epsinv_sizes_random_hpd(ng, rank, monkeypatch):
    # both forms of the panel and rank update (FP64 matrix cores, the default, and VALU)
    monkeypatch.setenv("XO_EPS_RANK", rank)
    say(f"epsinv random HPD ng={ng} rank update {rank}")
    X = random_complex(ng, (3 * ng + 2, ng))
    chi = -(X.conj().T @ X)[None] / (3 * ng)
    chi = np.concatenate([chi, 0.5 * chi])
    qpg = np.linspace(0.5, 3.0, ng)
    ref = epsinv_sym(chi, qpg)
    out = torch.empty(chi.shape, dtype=torch.complex128, device=DEV)
    xo.epsinv(_to(chi), qpg, out=out)
    assert rel_fro(out.cpu().numpy(), ref) < 1e-12
    # the deferred-check call gives the same result and all-zero flags
    info = torch.full((2,), -1, dtype=torch.int32, device=DEV)
    out2 = torch.empty_like(out)
    xo.epsinv(_to(chi), qpg, out=out2, info=info)
    assert torch.equal(out2, out) and info.tolist() == [0, 0]


def test_epsinv_not_positive_definite():
    ng = 40
    X = random_complex(3, (50, ng))
    chi = (X.conj().T @ X)[None] * 0.5          # positive: eps~ = I - s chi s is indefinite
    qpg = np.ones(ng)
    out = torch.empty(chi.shape, dtype=torch.complex128, device=DEV)
    with pytest.raises(xo.XoError) as e:
        xo.epsinv(_to(chi), qpg, out=out)
    assert e.value.code == xo.XO_ERR_NOTPD
    # deferred check: no error from the call, the flag lands in info
    info = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    xo.epsinv(_to(chi), qpg, out=out, info=info)
    assert info.item() > 0
    xo.epsinv(_to(chi), qpg, out=out, flags=xo.XO_EPS_LU_FALLBACK)
    s = np.sqrt(4 * np.pi) / qpg
    ref = np.linalg.inv(np.eye(ng) - s[:, None] * chi[0] * s[None, :])
    assert np.abs(out.cpu().numpy()[0] - ref).max() < 1e-9 * np.abs(ref).max()


def _chi_for_eps(M, qpg):
    """chi0 whose eps~ = I - s chi0 s is the given matrix M (per frequency)."""
    s = np.sqrt(4 * np.pi) / qpg
    return (np.eye(M.shape[-1])[None] - M) / (s[:, None] * s[None, :])[None]


@pytest.mark.parametrize("rank", ["valu", "mfma"])
@pytest.mark.parametrize("ng", [5, 64, 97, 200])
def test_epsinv_lu_fallback_pivots_inside_blocks(ng, rank, monkeypatch):
    """General (non-Hermitian) well-conditioned eps~ whose leading pivots are tiny or zero
    in the unpivoted order: frequency 0 has eps~_00 = 1e-14, frequency 1 has pairs of rows
    swapped inside each 64-block (zero diagonal where two rows meet), so elimination
    without pivoting fails or loses accuracy; the pivoted form matches numpy's LU inverse."""
    monkeypatch.setenv("XO_EPS_RANK", rank)
    say(f"epsinv LU fallback pivoting ng={ng} rank update {rank}")
    g = np.random.default_rng(ng)
    base = np.eye(ng) + 0.3 * (g.standard_normal((ng, ng)) + 1j * g.standard_normal((ng, ng))) / np.sqrt(ng)
    m0 = base.copy()
    m0[0, 0] = 1e-14
    perm = np.arange(ng)
    for i in range(0, ng - 1, 2):
        perm[i], perm[i + 1] = perm[i + 1], perm[i]
    m1 = np.eye(ng)[perm] @ (np.eye(ng) + 0.2 * (base - np.eye(ng)))
    M = np.stack([m0, m1])
    assert all(np.linalg.cond(m) < 500 for m in M)
    qpg = np.linspace(0.7, 2.5, ng)
    out = torch.empty(M.shape, dtype=torch.complex128, device=DEV)
    xo.epsinv(_to(_chi_for_eps(M, qpg)), qpg, out=out, flags=xo.XO_EPS_LU_FALLBACK)
    got = out.cpu().numpy()
    for j in range(2):
        ref = np.linalg.inv(M[j])
        assert np.linalg.norm(got[j] - ref) < 1e-11 * np.linalg.norm(ref), j


def test_epsinv_lu_fallback_reports_singular_block():
    """Invertible eps~ whose leading 64 x 64 block is zero: the blocked elimination does
    not pivot across blocks, so it reports XO_ERR_SINGULAR (or flags it in info) rather
    than returning a wrong inverse."""
    ng = 128
    M = np.zeros((1, ng, ng), complex)
    M[0, :64, 64:] = np.eye(64)
    M[0, 64:, :64] = np.eye(64)
    assert abs(np.linalg.det(M[0])) == 1.0
    qpg = np.ones(ng)
    out = torch.empty(M.shape, dtype=torch.complex128, device=DEV)
    with pytest.raises(xo.XoError) as e:
        xo.epsinv(_to(_chi_for_eps(M, qpg)), qpg, out=out, flags=xo.XO_EPS_LU_FALLBACK)
    assert e.value.code == xo.XO_ERR_SINGULAR
    info = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    xo.epsinv(_to(_chi_for_eps(M, qpg)), qpg, out=out, flags=xo.XO_EPS_LU_FALLBACK, info=info)
    assert info.item() == 1   # the first pivot of the first block


# ---------------------------------------------------------------------- end to end

# FP64 against the 1e-6 target, the split forms (FP32, bf16x3) against the 1e-4 target.
# Plain bf16 is not a split form (no correction): its element-wise rounding bounds are
# asserted by the chi0 and rho tests; here its measured eps~^-1 error on this small workload
# (a few hundred transitions average its operand rounding (at most 2^-8 each), about 3e-4) is held to 1e-3.
@pytest.mark.parametrize("name,prec,gate", [("c1", "fp64", 1e-6), ("c2_small", "fp64", 1e-6),
                                            ("c1", "fp32", 1e-4), ("c2_small", "fp32", 1e-4),
                                            ("c2_small", "bf16x3", 1e-4), ("c2_small", "bf16", 1e-3)])
def test_end_to_end(name, prec, gate):
    cr = crystal_for(name)
    say(f"end to end {name} {prec}")
    dc = DeviceCrystal.upload(cr, prec)
    M, dE, chi, E = run_crystal(dc)
    torch.cuda.synchronize()
    Eref, chiref = _oracle_eps(name)
    t = err_table(E.cpu().numpy(), Eref, chi.cpu().numpy(), chiref)
    say(f"  {t}")
    assert t["e_F"] <= gate
    if prec == "fp64":
        assert t["e_F"] < 1e-11


_ORC = {}


def _oracle_eps(name):
    if name not in _ORC:
        cr = crystal_for(name)
        chi = chi0_crystal(cr)
        _ORC[name] = (epsinv_sym(chi, crystal_qpg(cr)), chi)
    return _ORC[name]


def test_alloc_failure_is_reported_and_recovers():
    cr = crystal_for("c1_small")
    dc = DeviceCrystal.upload(cr, "fp64")
    xo.release_workspace()
    os.environ["XO_FAULT"] = "alloc"
    try:
        with pytest.raises(xo.XoError) as e:
            run_crystal(dc)
        assert e.value.code == xo.XO_ERR_ALLOC
    finally:
        del os.environ["XO_FAULT"]
    M, dE, chi, E = run_crystal(dc)
    Eref = epsinv_sym(chi0_crystal(cr), crystal_qpg(cr))
    assert rel_fro(E.cpu().numpy(), Eref) < 1e-11


# ------------------------------------------------------------- batched persistent

@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-5), ("bf16x3", 2e-4), ("bf16", None)])
@pytest.mark.parametrize("tune", [None, (1, 256, 2), (2, 512, 4), (2, 0, 8), (4, 256, 1), (4, 0, 0), (8, 0, 0),
                                  (8, 256, 1)])
def test_chi0_batch_uneven_items(prec, tol, tune):
    """Items with different G-set sizes and transition counts in one persistent launch."""
    if prec == "fp64" and tune is not None and tune[0] in (2, 4, 8):
        pytest.skip("two column tiles per wave and the block and strip forms exist for the bf16 forms only")
    if prec == "fp32" and tune is not None and tune[0] in (4, 8):
        pytest.skip("the block and strip forms exist for the bf16 forms only (a 2-tile tune runs the 1-tile form)")
    say(f"chi0 batch {prec} tune={tune}")
    shapes = [(700, 17), (1300, 33), (96, 50), (2000, 41)]
    w = [0.0, 0.3, 1.0]
    items, refs, bounds = [], [], []
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    for k, (nt, ng) in enumerate(shapes):
        M = random_complex(50 + k, (nt, ng))
        dE = random_positive(60 + k, nt, 0.05, 3.0)
        if prec != "fp64":
            M = M.astype(np.complex64).astype(np.complex128)
        refs.append(chi0_from_rho(M, dE, w, 0.5 + k))
        bounds.append(bf16_chi0_bound(M, dE, w, 0.5 + k) if tol is None else None)
        out = torch.empty((3, ng, ng), dtype=torch.complex128, device=DEV)
        items.append((_to(M, cdt), _to(dE, torch.float64), 0.5 + k, out))
    xo.chi0_batch(items, w, prec=prec, tune=tune)
    for (_, _, _, out), ref, bound in zip(items, refs, bounds):
        got = out.cpu().numpy()
        if tol is None:
            assert (np.abs(got - ref) / bound).max() <= 1.0
        else:
            assert rel_fro(got, ref) < tol
        for j in range(3):
            assert np.array_equal(got[j], got[j].conj().T)


def test_chi0_batch_equals_single_calls_and_autotune():
    shapes = [(900, 24), (1500, 40)]
    w = [0.0, 1.0]
    items = []
    for k, (nt, ng) in enumerate(shapes):
        M = random_complex(70 + k, (nt, ng))
        dE = random_positive(80 + k, nt, 0.05, 3.0)
        items.append((_to(M), _to(dE, torch.float64), 1.0, torch.empty((2, ng, ng), dtype=torch.complex128,
                                                                         device=DEV)))
    xo.chi0_batch(items, w)
    for Md, dEd, pref, out in items:
        single = torch.empty_like(out)
        xo.chi0(Md, dEd, w, pref, out=single)
        a, b = out.cpu().numpy(), single.cpu().numpy()
        assert np.abs(a - b).max() < 1e-14 * np.abs(b).max()
    best, ms = xo.chi0_autotune(items, w)
    say(f"  autotune best {best} {ms:.3f} ms")
    assert best[0] in (1, 2) and ms > 0
    xo.chi0_batch(items, w, tune=best)
    for Md, dEd, pref, out in items:
        single = torch.empty_like(out)
        xo.chi0(Md, dEd, w, pref, out=single)
        assert np.abs(out.cpu().numpy() - single.cpu().numpy()).max() < 1e-14 * single.abs().max().item()
