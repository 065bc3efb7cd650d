"""Shared helpers of the GPU tests: run a configuration on the GPU library
and on the FP64 oracle from the same seeded inputs and compare."""
import numpy as np
import torch

import oracle
import paper_0707_1581_amd as lbf

LATTICES = {"d3q19": oracle.D3Q19, "d2q9": oracle.D2Q9}
_A = {}


def weights(q=19):
    """a_i of the lattice with q populations, from the oracle's tables."""
    if q not in _A:
        _A[q] = oracle.tables(oracle.D3Q19 if q == 19 else oracle.D2Q9)[1]
    return _A[q]


def say(msg):
    print(msg, flush=True)


def oracle_params(cfg):
    keys = ("nx", "ny", "nz", "rho0", "kT", "gamma_bulk", "gamma_shear", "gamma_odd", "gamma_even", "seed")
    tm = cfg.get("thermal_modes", "all")
    return oracle.params(**{k: cfg[k] for k in keys if k in cfg},
                         thermal_modes=oracle.THERMAL_ALL if tm == "all" else oracle.THERMAL_STRESS_ONLY,
                         lattice=LATTICES[cfg.get("lattice", "d3q19")])


def scaled_err(got, want, rho0):
    """max over populations and sites of |n_gpu - n_oracle| / (a_i rho0)."""
    q = len(want)
    a = weights(q)
    d = np.abs(np.asarray(got, dtype=np.float64) - want)
    return float((d.reshape(q, -1).max(axis=1) / (a * rho0)).max())


def gpu_pops(lat):
    return lat.populations().double().cpu().numpy()
