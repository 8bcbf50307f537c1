"""Helpers shared by the GPU parity tests (CPU-side comparison only)."""
import numpy as np
import torch

import oracle

TOL = {"fp32": 1e-5, "bf16x3": 1e-5, "bf16": 2e-2}   # normwise vs the FP64 oracle
EMU_TOL = 1e-6                                       # normwise vs precision emulation


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def as_em(out, layout):
    """GPU output as (K, E, Np) float64 numpy array."""
    o = out.detach().cpu().numpy().astype(np.float64)
    return o if layout == "em" else np.ascontiguousarray(o.transpose(0, 2, 1))


def check_against_oracle(D, u, out_em, layout, precision, e0=0):
    """Normwise errors of an (K, ne, Np) GPU chunk vs the FP64 oracle and vs
    the oracle's emulation of the precision; asserts both tolerances."""
    ne = out_em.shape[1]
    ref = oracle.contract(D, u, layout, "fp32", e0, ne)
    err = oracle.rel_err(out_em, ref)
    assert err <= TOL[precision], (precision, err)
    if precision != "fp32":
        emu = oracle.contract(D, u, layout, precision, e0, ne)
        err_emu = oracle.rel_err(out_em, emu)
        assert err_emu <= EMU_TOL, (precision, err_emu)
    return err
