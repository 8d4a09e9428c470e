"""Mutation check of the oracle's pins: each plausible mistake planted in a
copy of the oracle source (on the CPU) must be caught by at least one pin."""
import os
import shutil

import pytest

from oracle import oracle as O
from tests import pins

SRC = os.path.join(os.path.dirname(O.__file__), "gs_oracle.c")

MUTATIONS = {
    "uvv_sign_in_u": ("double du = (Du * lapu - uvv)", "double du = (Du * lapu + uvv)"),
    "uvv_sign_in_v": ("(Dv * lapv + uvv)", "(Dv * lapv - uvv)"),
    "uvv_both_signs": ("double du = (Du * lapu - uvv) + F * (1.0 - uc);\n",
                       "double du = (Du * lapu + uvv) + F * (1.0 - uc); uvv = -uvv;\n"),
    "uvv_power": ("uc * (vc * vc)", "uc * vc"),
    "feed_sign": ("F * (1.0 - uc)", "F * (1.0 + uc)"),
    "feed_dropped_in_kill": ("(F + k) * vc", "k * vc"),
    "Dv_is_Du": ("(Dv * lapv + uvv)", "(Du * lapv + uvv)"),
    "x_plus_wrong": ("xp = (x + 1) % nx", "xp = (x + 2) % nx"),
    "y_minus_wrong": ("ym = (y + ny - 1) % ny", "ym = y"),
    "z_pair_wrong": ("double sz = AT(x, y, zm) + AT(x, y, zp);", "double sz = AT(x, y, zm) + AT(x, y, zm);"),
    "divide_by_7": ("(s - 6.0 * c) / 6.0", "(s - 6.0 * c) / 7.0"),
    "centre_weight_5": ("(s - 6.0 * c) / 6.0", "(s - 5.0 * c) / 6.0"),
    "dt_dropped": ("un[c] = uc + du * dt;", "un[c] = uc + du;"),
    "noise_wrong_step": ("gso_noise_r(seed, t, (uint64_t)c)", "gso_noise_r(seed, t + 1, (uint64_t)c)"),
    "noise_without_half": ("((double)w + 0.5)", "((double)w)"),
    "noise_word_index": ("out[idx & 3u]", "out[idx & 1u]"),
    "philox_weyl_swapped": ("k0 += PHILOX_W0;", "k0 += PHILOX_W1;"),
    "philox_nine_rounds": ("round < 10", "round < 9"),
    "cube_corner_off_by_one": ("int x0 = (nx - side) / 2", "int x0 = (nx - side + 1) / 2"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    mutated = tmp_path / "gs_oracle_mut.c"
    mutated.write_text(src.replace(old, new, 1))
    lib = O.OracleLib(O.build_from(str(mutated), str(tmp_path / "libmut.so")))
    caught = []
    for check in pins.ALL:
        try:
            check(impl=lib)
        except AssertionError:
            caught.append(check.__name__)
    assert caught, f"no pin catches mutation {name}"
