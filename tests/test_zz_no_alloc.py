"""xo_epsinv_noalloc (static scratch, no allocation) against xo_epsinv, through the C ABI."""

import ctypes as C
import os

import numpy as np
import pytest
import torch

from synth.rand import random_complex  # noqa: E402
from paper_1902_03837_amd import xo  # noqa: E402

DEV = "cuda"

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    xo.lib()


def _hpd_chi(ng, nw, seed):
    X = random_complex(seed, (2 * ng + 3, ng))
    base = -(X.conj().T @ X) / (2 * ng)
    return np.stack([base * (1.0 / (1 + j)) for j in range(nw)])


def test_noalloc_equals_epsinv_twice_second_smaller():
    # two calls in a row on the shared scratch, the second with a smaller input; each
    # against xo_epsinv on the same input (same kernels: bitwise equal)
    for ng, nw, flags in ((200, 5, xo.XO_EPS_SYM), (97, 2, xo.XO_EPS_NONSYM)):
        say(f"noalloc ng={ng} nw={nw} flags={flags}")
        chi = torch.from_numpy(_hpd_chi(ng, nw, ng)).to(DEV)
        qpg = np.linspace(0.6, 2.8, ng)
        ref = torch.empty_like(chi)
        got = torch.full_like(chi, complex(7.0, 7.0))
        xo.epsinv(chi, qpg, out=ref, flags=flags)
        xo.epsinv(chi, qpg, out=got, flags=flags, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)


def test_noalloc_flags_and_fallback():
    say("noalloc NOTPD, deferred flags, LU fallback")
    ng = 40
    X = random_complex(3, (50, ng))
    chi = torch.from_numpy(((X.conj().T @ X)[None] * 0.5)).to(DEV)   # eps~ indefinite
    qpg = np.ones(ng)
    out = torch.empty_like(chi)
    with pytest.raises(xo.XoError) as e:
        xo.epsinv(chi, qpg, out=out, noalloc=True)
    assert e.value.code == xo.XO_ERR_NOTPD
    info = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    xo.epsinv(chi, qpg, out=out, info=info, noalloc=True)
    assert info.item() > 0
    ref = torch.empty_like(chi)
    xo.epsinv(chi, qpg, out=ref, flags=xo.XO_EPS_LU_FALLBACK)
    xo.epsinv(chi, qpg, out=out, flags=xo.XO_EPS_LU_FALLBACK, noalloc=True)
    assert torch.equal(out, ref)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    ng, nw = 3000, 16     # 3000 x 16 x 1024 bytes of panel = 49 MB: fits
    assert 1024 * ng * nw < (64 << 20)
    ng, nw = 3000, 32     # 98 MB: does not
    chi = torch.zeros((1, 1, 1), dtype=torch.complex128, device=DEV)
    a = xo.EpsArgs()
    a.ng, a.nw = ng, nw
    qpg = np.ones(ng)
    a.qpg, a.chi0, a.out, a.flags = qpg.ctypes.data_as(C.POINTER(C.c_double)), chi.data_ptr(), chi.data_ptr() + 16, 0
    rc = xo.lib().xo_epsinv_noalloc(C.byref(a), None)
    assert rc == xo.XO_ERR_UNSUPPORTED and b"scratch" in xo.lib().xo_last_error()
