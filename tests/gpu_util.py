"""Helpers shared by the GPU parity tests (CPU-side comparison only)."""
import numpy as np
import torch

import oracle

TOL = {"fp32": 1e-5, "bf16x3": 1e-5, "bf16": 2e-2}   # normwise vs the FP64 oracle
EMU_TOL = 1e-6                                       # normwise vs precision emulation


def emu_tol(n):
    """Normwise tolerance against the oracle's emulation of the same
    precision: only FP32 accumulation separates the two, whose error grows
    like sqrt(n) * 2^-24 for n-term sums.  A wrong split or a missing bf16x3
    term shows up at ~1e-3."""
    return max(EMU_TOL, 8.0 * n ** 0.5 * 2.0 ** -24)


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def as_em(out, layout):
    """GPU output as (K, E, Np) float64 numpy array."""
    o = out.detach().cpu().numpy().astype(np.float64)
    return o if layout == "em" else np.ascontiguousarray(o.transpose(0, 2, 1))


# Componentwise error bound of one product under bf16x3: the dropped lo*lo
# term and the residuals x - hi - lo are each below 2^-16 of |a||b|.
BF16X3_PRODUCT_BOUND = 3 * 2.0 ** -16
SHORT_REDUCTION = 32   # below this, errors do not average: use the bound


def assert_within_bound(y, ref, absref, n, precision):
    """|y - ref| <= (per-product bound + FP32 accumulation) * sum|a||b|."""
    per = {"bf16x3": BF16X3_PRODUCT_BOUND, "fp32": 0.0, "bf16": 2.0 ** -7}[precision]
    bound = (per + n * 2.0 ** -24) * absref + 1e-30
    assert np.all(np.abs(y - ref) <= bound), (precision, float(np.max(np.abs(y - ref) / bound)))


def check_against_oracle(D, u, out_em, layout, precision, e0=0):
    """Normwise errors of an (K, ne, Np) GPU chunk vs the FP64 oracle and vs
    the oracle's emulation of the precision; asserts both tolerances.  For
    bf16x3 with fewer than 32 terms per sum the componentwise per-product
    bound is asserted as well (there is no averaging to rely on there)."""
    ne = out_em.shape[1]
    ref = oracle.contract(D, u, layout, "fp32", e0, ne)
    err = oracle.rel_err(out_em, ref)
    Np = D.shape[1]
    if precision == "bf16x3" and Np < SHORT_REDUCTION:
        absref = oracle.contract(np.abs(D), np.abs(u), layout, "fp32", e0, ne)
        assert_within_bound(out_em, ref, absref, Np, precision)
    assert err <= TOL[precision], (precision, err)
    if precision != "fp32":
        emu = oracle.contract(D, u, layout, precision, e0, ne)
        err_emu = oracle.rel_err(out_em, emu)
        assert err_emu <= emu_tol(Np), (precision, err_emu)
    return err
