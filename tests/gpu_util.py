"""Shared helpers of the GPU tests: run a configuration on the GPU library
and on the FP64 oracle from the same seeded inputs and compare."""
import numpy as np
import torch

import oracle
import paper_0707_1581_amd as lbf

A = None


def weights():
    global A
    if A is None:
        A = oracle.tables()[1]
    return A


def say(msg):
    print(msg, flush=True)


def oracle_params(cfg):
    keys = ("nx", "ny", "nz", "rho0", "kT", "gamma_bulk", "gamma_shear", "gamma_odd", "gamma_even", "seed")
    tm = cfg.get("thermal_modes", "all")
    return oracle.params(**{k: cfg[k] for k in keys if k in cfg},
                         thermal_modes=oracle.THERMAL_ALL if tm == "all" else oracle.THERMAL_STRESS_ONLY)


def scaled_err(got, want, rho0):
    """max over populations and sites of |n_gpu - n_oracle| / (a_i rho0)."""
    a = weights()
    d = np.abs(np.asarray(got, dtype=np.float64) - want)
    return float((d.reshape(19, -1).max(axis=1) / (a * rho0)).max())


def gpu_pops(lat):
    return lat.populations().double().cpu().numpy()
