"""Save and load a generated crystal (plain arrays in an .npz, no pickled objects), so that
several runs of one session can share an expensive fixture such as the large cell."""

from __future__ import annotations

import json
import os

import numpy as np

from .crystal import Crystal, Lattice


def save_crystal(cr: Crystal, path: str) -> None:
    arrs = dict(avec=cr.lat.avec, bvec=cr.lat.bvec, lat_scalars=np.array([cr.lat.omega, cr.lat.unit]),
                kf=cr.kf, qf=cr.qf, grid=np.array(cr.grid), gmill=cr.gmill, omegas=cr.omegas,
                pair_idx=np.array([[ik, ikp] for ik, ikp, _ in cr.pairs]),
                pair_g0=np.array([g0 for _, _, g0 in cr.pairs]))
    for i, (m, c, e) in enumerate(zip(cr.mill, cr.coef, cr.eps)):
        arrs[f"mill{i}"], arrs[f"coef{i}"], arrs[f"eps{i}"] = m, c, e
    meta = dict(ecut=cr.ecut, nocc=cr.nocc, scissor=cr.scissor, seed=cr.seed, nk=len(cr.mill),
                nocc_k=cr.nocc_k, meta=cr.meta)
    arrs["json"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrs)
    os.replace(tmp, path)


def load_crystal(path: str) -> Crystal:
    z = np.load(path, allow_pickle=False)
    meta = json.loads(bytes(z["json"]).decode())
    nk = meta["nk"]
    lat = Lattice(z["avec"], z["bvec"], float(z["lat_scalars"][0]), float(z["lat_scalars"][1]))
    pairs = [(int(a), int(b), g.astype(np.int32)) for (a, b), g in zip(z["pair_idx"], z["pair_g0"])]
    return Crystal(lat=lat, kf=z["kf"], qf=z["qf"], grid=tuple(int(x) for x in z["grid"]), ecut=meta["ecut"],
                   nocc=meta["nocc"], mill=[z[f"mill{i}"] for i in range(nk)], coef=[z[f"coef{i}"] for i in range(nk)],
                   eps=[z[f"eps{i}"] for i in range(nk)], gmill=z["gmill"], omegas=z["omegas"], pairs=pairs,
                   scissor=meta["scissor"], seed=meta["seed"], meta=meta["meta"], nocc_k=meta["nocc_k"])


def cached_crystal(name: str, cache_dir=None, progress=None, seed=None):
    """crystal_for(name, seed), kept in cache_dir/<name>[_s<seed>].npz when a directory is given."""
    from .configs import crystal_for
    if cache_dir:
        path = os.path.join(cache_dir, f"{name}.npz" if seed is None else f"{name}_s{seed}.npz")
        if os.path.exists(path):
            return load_crystal(path)
    cr = crystal_for(name, seed=seed, progress=progress)
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
        save_crystal(cr, path)
    return cr
