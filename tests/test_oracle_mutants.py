"""Each planted oracle mistake is caught by the pins (mutation testing, CPU only).

The mistakes are compiled into throw-away builds of the oracle (OR_MUTANT=k);
the shipped oracle is built without them."""
import os

import pytest

import oracle
from oracle import build as obuild

import pins

MUTANTS = {
    1: ("dropped z term of r2", [pins.check_pair_distance]),
    2: ("no periodic minimum image", [pins.check_periodic]),
    3: ("inclusive cutoff r2 <= rc2", [pins.check_cutoff_strict]),
    5: ("no one-A-per-T selection", [pins.check_two_a_one_t]),
    7: ("acceptance probability doubled", [pins.check_isolated_cluster_probability,
                                           pins.check_acceptance_ratio]),
    9: ("bonded pairs not excluded", [pins.check_exclusion]),
    10: ("state deltas swapped between roles", [pins.check_chain_transfer]),
    12: ("off-centre jitter offsets", [pins.check_jitter_distribution]),
    14: ("FP64 recheck without the periodic wrap", [pins.check_near_cutoff]),
    15: ("FP64 tolerance applied to r^2", [pins.check_near_cutoff]),
    16: ("FP64 recheck counts every particle as an A", [pins.check_near_cutoff]),
    17: ("FP32 side of the recheck evaluated in FP64", [pins.check_near_cutoff_disagree]),
    18: ("nearest: bonded pairs stay candidates", [pins.check_nearest_exclusion_first]),
    19: ("nearest: pairs need not be mutual", [pins.check_nearest_mutual]),
    20: ("kinetics: partners counted under the T's state", [pins.check_kinetics_hand]),
    21: ("several rules: no cross-role selection (step 8)", [pins.check_multi_cross_role]),
    22: ("mirror-LJ force with the wrong sign", [pins.check_md_two_body]),
}


@pytest.mark.parametrize("k", sorted(MUTANTS))
def test_mutant_is_caught(k, tmp_path):
    path = obuild.build(out=os.path.join(str(tmp_path), "liboracle_m%d.so" % k),
                        extra=("-DOR_MUTANT=%d" % k,))
    lib = oracle.load(path)
    what, checks = MUTANTS[k]
    for check in checks:
        with pytest.raises(AssertionError):
            check(lib)
