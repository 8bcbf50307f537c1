"""Mistakes planted in copies of the oracle (on the CPU) must each fail at
least one pin: evidence that the pins pin the oracle, not just re-run it."""
import os

import pytest

import oracle
from oracle.build import SRC, build
from tests import oracle_pins

# (name, exact text in oracle.c, replacement)
MUTANTS = [
    ("transposed_D", "acc += prod(Dk[(long)i * Np + j]", "acc += prod(Dk[(long)j * Np + i]"),
    ("dropped_first_term", "for (int j = 0; j < Np; ++j) {", "for (int j = 1; j < Np; ++j) {"),
    ("dm_index_as_em", ": u[(long)j * E + e];", ": u[e * Np + j];"),
    ("sign_flip", "acc += prod(", "acc -= prod("),
    ("bf16x3_drops_hi_lo", "(double)ah * (double)bl +", ""),
    ("bf16x3_lo_lo_instead_of_lo_hi", "(double)al * (double)bh;", "(double)al * (double)bl;"),
    ("truncating_round", "if (low > 0x8000u || (low == 0x8000u && lsb)) keep += 0x10000u;", "(void)lsb;"),
    ("ties_away", "(low == 0x8000u && lsb)", "(low == 0x8000u)"),
    ("gemm_B_transposed", "prod(a, Brow[n], precision)", "prod(a, B[n * Kd + k], precision)"),
    ("gemm_drops_last_k", "for (long k = 0; k < Kd; ++k) {", "for (long k = 0; k < Kd - 1; ++k) {"),
    ("bf16_keeps_fp32", "return (double)oracle_bf16_rne(a) * (double)oracle_bf16_rne(b);",
     "return (double)a * (double)b;"),
    ("chunk_offset_ignored", "long e = e0 + de;", "long e = de;"),
    ("dg_G_transposed", "G[(e * K + d) * K + k]", "G[(e * K + k) * K + d]"),
    ("dg_dm_G_index_as_em", "G[((long)d * K + k) * E + e]", "G[(e * K + d) * K + k]"),
    ("dg_wrong_derivative", "acc += (double)g * t[k * Np + i];", "acc += (double)g * t[d * Np + i];"),
    ("dg_drops_last_k", "for (int k = 0; k < K; ++k) {\n                    float g",
     "for (int k = 0; k < K - 1; ++k) {\n                    float g"),
    ("surface_face_index", "long c = m / nfp;", "long c = m / nf;"),
    ("surface_scale_ignored", "float g = sv * fv;", "float g = fv; (void)sv;"),
    ("surface_scale_in_double", "acc += prod(L[(long)i * M + m], g, precision);",
     "acc += (double)L[(long)i * M + m] * ((double)sv * (double)fv);"),
    ("surface_L_transposed", "prod(L[(long)i * M + m], g, precision)",
     "prod(L[(long)m * Np + i], g, precision)"),
    ("surface_dm_flux_as_em", ": f[m * E + e];", ": f[e * M + m];"),
    ("coulomb_no_sqrt", "if (r2 > 0.0) acc += q / sqrt(r2);", "if (r2 > 0.0) acc += q / r2;"),
    ("coulomb_sum_not_difference", "double d = xt[c] - ys;", "double d = xt[c] + ys;"),
    ("coulomb_self_pair_kept", "if (r2 > 0.0) acc += q / sqrt(r2);",
     "acc += q / sqrt(r2 + 1e-300);"),
    ("coulomb_soa_stride", "(double)sr[c * ns + s]", "(double)sr[c * nt + s]"),
    ("coulomb_charge_field", "(double)sr[4 * s + 3]", "(double)sr[4 * s + 2]"),
    ("coulomb_chunk_offset", "long t = t0 + dt;", "long t = dt;"),
    ("dg_G_in_float", "acc += (double)g * t[k * Np + i];", "acc += (double)(g * (float)t[k * Np + i]);"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_fails_a_pin(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    lib = build(src=str(mut), out=str(tmp_path / "liboracle_mut.so"))
    o = oracle.Oracle(lib)
    failed = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(o)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
