"""Seeded random numbers for synthetic inputs (numpy PCG64)."""

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_complex(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    """Complex128 array with independent N(0, scale^2/2) real and imaginary parts."""
    g = rng(seed)
    s = scale / np.sqrt(2.0)
    return (g.normal(0.0, s, shape) + 1j * g.normal(0.0, s, shape)).astype(np.complex128)


def random_positive(seed: int, n: int, lo: float, hi: float) -> np.ndarray:
    return rng(seed).uniform(lo, hi, n).astype(np.float64)


def mlp_init(dims, seed):
    """Initial MLP parameters: W_l ~ U(-a, a), a = sqrt(6 / fan_in), b_l = 0 (FP64 arrays)."""
    g = rng(seed)
    out = []
    for din, dout in zip(dims[:-1], dims[1:]):
        a = np.sqrt(6.0 / din)
        out.append((g.uniform(-a, a, (dout, din)), np.zeros(dout)))
    return out


def flatten_params(params) -> np.ndarray:
    """Per layer W [out][in] row-major then b [out], as one FP32 vector."""
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in params]).astype(np.float32)


def device_random_rho(seed: int, nt: int, ng: int, dtype, device, scale: float = 0.02):
    """Seeded complex strengths [nt][ng] and pole energies [nt] (uniform in [0.05, 5.05) Ha)
    generated on the device by torch's counter-based generator, for inputs too large to build
    on the host (a full large-cell transition set). Real and imaginary parts ~ N(0, scale^2/2)."""
    import torch
    g = torch.Generator(device=device).manual_seed(seed)
    M = torch.randn((nt, ng), dtype=dtype, device=device, generator=g) * scale
    dE = torch.rand(nt, dtype=torch.float64, device=device, generator=g) * 5.0 + 0.05
    return M, dE
