"""The pins must catch plausible mistakes: each planted mistake (built into a
separate copy of the oracle with -DORC_MUTANT=k, on the CPU) has to fail at
least one pin of tests/test_oracle_pins.py."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    1: ("dropped lambda div-div term (elasticity)", "elasticity"),
    2: ("wrong sign of the F^{-T} derivative (hyperelastic tangent)", "hyper"),
    3: ("transposed K in the physical gradient", "helmholtz or elasticity"),
    4: ("wrong index phi_i phi_i in the mass integrand", "mass"),
    5: ("Gauss-Jacobi weights off by a factor 2", "rule"),
    6: ("wrong denominator in the Silvester factor", "basis"),
    7: ("dropped lambda ln J term of the tangent", "hyper"),
    8: ("coefficient function evaluated with a shifted basis index", "coefficients"),
    9: ("only the first pre-multiplying coefficient function applied", "coefficients"),
    10: ("element matrix inserted transposed", "global assembly"),
    11: ("last local column dropped from the insertion", "global assembly"),
    12: ("non-affine prism geometry taken at the centroid for every point", "non-affine geometry"),
    13: ("test and trial basis indices swapped in a generic term", "generic forms"),
    14: ("curved-simplex geometry taken at the first point for every point", "curved geometry"),
    15: ("component blocks of a vector-valued form transposed", "generic vector forms"),
}

PINS = {
    1: "elasticity_exact_rational or elasticity_p1_textbook",
    2: "hyper_tangent_is_residual_derivative",
    3: "mass_and_helmholtz_exact_rational",
    4: "mass_p1_triangle_closed_form or mass_and_helmholtz_exact_rational",
    5: "rule_exact_to_degree",
    6: "basis_kronecker",
    7: "hyper_tangent_is_residual_derivative",
    8: "coefficient_fields_exact_rational",
    9: "coefficient_fields_exact_rational or coefficient_fields_invariants",
    10: "pattern_and_insert_brute_force",
    11: "global_quadratic_forms_exact or pattern_and_insert_brute_force",
    12: "zjittered_box_quadratic_forms",
    13: "spec_constant_terms_exact",
    14: "one_curved_edge_volume or curved_box_quadratic_forms",
    15: "vspec_blocks_exact",
}

# pins of the global assembly live in their own module
PIN_FILE = {10: "test_global_pins.py", 11: "test_global_pins.py", 12: "test_nonaffine_pins.py",
            13: "test_form_spec_pins.py", 14: "test_curved_pins.py", 15: "test_form_spec_pins.py"}


@pytest.mark.parametrize("k", sorted(MUTANTS))
def test_pins_catch_planted_mistake(k):
    with tempfile.TemporaryDirectory() as tmp:
        lib = oracle.build(force=True, out=os.path.join(tmp, f"liboracle_m{k}.so"), defines=[f"ORC_MUTANT={k}"])
        env = dict(os.environ, FE_ORACLE_LIB=lib)
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", PIN_FILE.get(k, "test_oracle_pins.py")), "-k", PINS[k]],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode == 1 and "failed" in r.stdout, (MUTANTS[k], r.stdout[-2000:])
