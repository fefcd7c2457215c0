"""Planted mistakes in the oracle must each fail at least one pin.

Every mutant is the oracle source compiled with -DDHO_MUTANT=k, which plants
one plausible mistake (dropped term, wrong sign, transposed cell, wrong loop
bound, wrong rounding, wrong bin edge, wrong histogram order, missing image
search, wrong scale). Runs on the CPU only."""
import os
import tempfile

import pytest

import oracle
import pins

MUTANTS = {
    1: "q drops the z component",
    2: "minimum image adds the shift instead of subtracting it",
    3: "cell read as columns (transposed)",
    4: "single-species loop includes j == i",
    5: "bin index rounds instead of truncating",
    6: "upper range edge closed (t <= n_bins)",
    7: "minimum image rounds by truncation",
    8: "cross-species histograms ordered first",
    9: "image search never runs",
    10: "triclinic inverse keeps only its diagonal",
    11: "scale r_max/n_bins instead of n_bins/r_max",
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_mutant_is_caught(mutant, tmp_path):
    path = oracle.build(mutant=mutant, out=str(tmp_path / f"libdh_oracle_m{mutant}.so"))
    lib = oracle.load(path=path)
    assert lib.dho_mutant() == mutant
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(lib)
        except AssertionError as e:
            failed.append(f"{pin.__name__}: {e}")
    assert failed, f"mutant {mutant} ({MUTANTS[mutant]}) passed every pin"
