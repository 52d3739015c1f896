"""Planted mistakes in copies of the oracle, caught by its pins.

Each case copies oracle/acs_oracle.c, makes one plausible mistake in the
copy (a permutation applied the wrong way round, a dropped term, a wrong
index), builds it into a temporary library and runs the pins of
tests/test_oracle_rl.py against it: at least one pin must fail.  This shows
the pins would notice such a mistake in the oracle itself.  Nothing here
touches the built oracle or the GPU library.
"""
from __future__ import annotations

import os
import subprocess

import pytest

from oracle import oracle as O

import test_oracle_rl as R

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "acs_oracle.c")

# (name, text in the oracle, replacement): each text must occur exactly once
MUTANTS = [
    ("permute gathers with inv_perm",
     "s->Q0[4 * p + c] = s->P[4 * s->perm[p] + c];",
     "s->Q0[4 * p + c] = s->P[4 * s->inv_perm[p] + c];"),
    ("integrate un-permutes with perm",
     "int32_t p = s->inv_perm[i];",
     "int32_t p = s->perm[i];"),
    ("integrate reads the predicted row of place i",
     "float x = s->Q0[4 * p + c];",
     "float x = s->Q0[4 * i + c];"),
    ("velocity update drops the correction",
     "float v = s->V[4 * i + c] + (x - s->P[4 * i + c]) / s->dt;",
     "float v = s->V[4 * i + c];"),
    ("inverse permutation stores the place of the wrong body",
     "s->perm[pos] = b; s->inv_perm[b] = pos; pos++;",
     "s->perm[pos] = b; s->inv_perm[pos] = b; pos++;"),
]

PINS = [R.pin_permute_groups_islands, R.pin_integrate_unpermutes_without_sweeps,
        R.pin_free_bodies_fly_free_in_a_full_step, R.pin_pair_velocity_from_correction]


def build_mutant(tmp_path, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"oracle source changed: {old!r} not found exactly once"
    src = tmp_path / "acs_oracle_mutant.c"
    src.write_text(text.replace(old, new))
    hdr = os.path.join(os.path.dirname(SRC))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-I", hdr, "-o", str(lib), str(src), "-lm"], check=True, capture_output=True)
    return O.load(str(lib))


def test_pins_pass_on_the_oracle():
    for pin in PINS:
        pin()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    L = build_mutant(tmp_path, old, new)
    failed = []
    for pin in PINS:
        try:
            pin(L)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin fails with the mistake '{name}'"
