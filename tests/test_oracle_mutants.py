"""The oracle's pins must catch plausible mistakes.  Each case builds the
oracle with one planted mistake (a dropped term, a wrong sign, a wrong or
transposed index, swapped operands) and reruns the pins that should see it,
in a subprocess, expecting them to fail."""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CASES = {
    1: ("dropped up-neighbour term in the local field",
        ["test_oracle_model.py::test_metropolis_samples_boltzmann_L4",
         "test_oracle_model.py::test_tracked_energy_equals_recomputed_after_annealing"]),
    2: ("wrong sign of the energy shift in ln Q",
        ["test_oracle_resample.py::test_counts_are_floor_or_ceil_of_mean"]),
    3: ("wrong row index of the upper bond coupling",
        ["test_oracle_physics.py::test_gauge_symmetry_of_pmJ_model"]),
    4: ("acceptance thresholds of dE=4 and dE=8 swapped",
        ["test_oracle_model.py::test_metropolis_samples_boltzmann_L4"]),
    5: ("transposed index of the right neighbour in the energy",
        ["test_oracle_model.py::test_energy_matches_bond_sum"]),
    6: ("level multiplicity dropped from the weight sum",
        ["test_oracle_resample.py::test_counts_are_floor_or_ceil_of_mean"]),
    7: ("ln Omega dropped from the free energy",
        ["test_oracle_physics.py::test_lnZ_and_Zhat_unbiased_L4"]),
    8: ("the -rho term dropped from the Poisson probabilities",
        ["test_oracle_poisson.py::test_draw_inverts_the_poisson_cdf"]),
    9: ("the ground-state energy term dropped from the heating start's ln Z",
        ["test_oracle_heating.py::test_heating_lnZ_L4_matches_enumeration"]),
    10: ("sign of the Potts energy change flipped",
         ["test_oracle_potts.py::test_metropolis_samples_boltzmann_q3_L4"]),
    11: ("systematic comb read over the wrong interval",
         ["test_oracle_systematic.py::test_counts_are_floor_or_ceiling_and_size_is_exact"]),
    12: ("multinomial draws counted from the current size, not the target",
         ["test_oracle_systematic.py::test_multinomial_draws_follow_the_weights"]),
    13: ("max instead of min of the two distributions in the overlap",
         ["test_oracle_overlap.py::test_overlap_equals_the_per_replica_form"]),
    14: ("bisection returns the end that misses the target",
         ["test_oracle_overlap.py::test_bisection_inverts_the_two_level_overlap"]),
    15: ("one factor of beta dropped from the specific heat",
         ["test_oracle_physics.py::test_observables_L4_match_enumeration"]),
    16: ("the 1/R dropped from the entropic family size",
         ["test_oracle_families.py::test_family_stats_closed_forms"]),
    17: ("a copy takes its parent's slot instead of its parent's family",
         ["test_oracle_families.py::test_families_compose_over_resamplings"]),
    18: ("every colour site of a plane group reads the same plane bits",
         ["test_oracle_rng_planes.py::test_plane_draws_are_fair_and_independent",
          "test_oracle_rng_planes.py::test_planes_metropolis_samples_boltzmann_L4"]),
    19: ("the excited states dropped from the heating start's ln Z",
         ["test_oracle_heating.py::test_start_lnZ_ising_L4_within_the_expansion_bound",
          "test_oracle_heating.py::test_start_lnZ_potts_q3_L4_within_the_expansion_bound"]),
}


@pytest.mark.parametrize("mutant", sorted(CASES))
def test_planted_mistake_is_caught(mutant, tmp_path):
    what, pins = CASES[mutant]
    so = str(tmp_path / ("liboracle_m%d.so" % mutant))
    oracle.build(mutant=mutant, out=so)
    env = dict(os.environ, PA_ORACLE_SO=so)
    for pin in pins:
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q",
                            os.path.join(HERE, pin)], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=300)
        assert r.returncode != 0, "mutant %d (%s) passed %s" % (mutant, what,
                                                               pin)
