"""The pins catch plausible mistakes: each case plants one slip in a copy of the
oracle source (on the CPU), builds it, runs the pin that should notice, and
expects that pin to fail.  The unmodified oracle passes every one of these pins
in its own test module."""
import gc
import os

import pytest

from oracle import oracle as O
from tests import test_oracle_cfl as T_cfl
from tests import test_oracle_fallback as T_fb
from tests import test_oracle_flux_quadrature as T_fq

SLIPS = {
    # the initial parts' micro-slope weight q4 with the wrong sign
    "q4_sign": ("q4 = -2.0 * tau * tau + tau * (d + 2.0 * tau) * E;",
                "q4 = 2.0 * tau * tau + tau * (d + 2.0 * tau) * E;",
                lambda: T_fq.test_flux_matches_quadrature_of_the_interface_distribution(1.0)),
    # the equilibrium part's slope weight q1 with the wrong sign
    "q1_sign": ("q1 = 2.0 * tau * tau - tau * d - tau * (d + 2.0 * tau) * E;",
                "q1 = -2.0 * tau * tau + tau * d + tau * (d + 2.0 * tau) * E;",
                lambda: T_fq.test_flux_matches_quadrature_of_the_interface_distribution(0.1)),
    # the spatial-slope moment of the left initial part dropped
    "drop_e1": ("el[1][a] += al[j][b] * expect(&Mlp, &P_UUPP[j][b][a]);",
                "el[1][a] += 0.0 * al[j][b];",
                T_fq.test_equal_states_give_the_navier_stokes_distribution),
    # the collision takes the wrong half spaces (hook and flux)
    "collision_halves": ("make_moments(sl.U, sl.V, sl.W, sl.lam, K, +1, &Mlp);\n"
                         "    make_moments(sr.U, sr.V, sr.W, sr.lam, K, -1, &Mrn);\n"
                         "    for (int a = 0; a < 5; ++a) q0[a]",
                         "make_moments(sl.U, sl.V, sl.W, sl.lam, K, -1, &Mlp);\n"
                         "    make_moments(sr.U, sr.V, sr.W, sr.lam, K, +1, &Mrn);\n"
                         "    for (int a = 0; a < 5; ++a) q0[a]",
                         T_fq.test_collision_of_unequal_states_matches_quadrature),
    "flux_collision_halves": ("make_moments(sl.U, sl.V, sl.W, sl.lam, K, +1, &Mlp);\n"
                              "    make_moments(sr.U, sr.V, sr.W, sr.lam, K, -1, &Mrn);\n"
                              "    /* compatibility",
                              "make_moments(sl.U, sl.V, sl.W, sl.lam, K, -1, &Mlp);\n"
                              "    make_moments(sr.U, sr.V, sr.W, sr.lam, K, +1, &Mrn);\n"
                              "    /* compatibility",
                              lambda: T_fq.test_flux_matches_quadrature_of_the_interface_distribution(0.0)),
    # the equilibrium slope from the sum rather than the mean of the two sides
    "dq0_sum": ("b0[q] = 0.5 * (dQl[j][q] + dQr[j][q]) / s0.rho;",
                "b0[q] = (dQl[j][q] + dQr[j][q]) / s0.rho;",
                lambda: T_fq.test_flux_matches_quadrature_of_the_interface_distribution(0.0)),
    # the fallback variant that keeps the physical side's gradient
    "fallback_one_side": ("gl[q][0] = gl[q][1] = gl[q][2] = 0.0;\n        gr[q][0] = gr[q][1] = gr[q][2] = 0.0;",
                          "if (!okl) gl[q][0] = gl[q][1] = gl[q][2] = 0.0;\n"
                          "        if (!okr) gr[q][0] = gr[q][1] = gr[q][2] = 0.0;",
                          T_fb.test_fallback_rule_is_first_order_at_the_point),
    # the CFL length as the inradius instead of the inscribed-sphere diameter
    "cfl_radius": ("m->hdt[c] = 6.0 * m->vol[c] / asum[c];",
                   "m->hdt[c] = 3.0 * m->vol[c] / asum[c];",
                   T_cfl.test_cfl_length_is_inscribed_sphere_diameter),
}


@pytest.mark.parametrize("slip", sorted(SLIPS))
def test_pin_catches_planted_slip(slip, tmp_path):
    old, new, pin = SLIPS[slip]
    src = open(O.SRC).read()
    assert src.count(old) == 1, f"the slip site of {slip} is no longer in the oracle source"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    mutant = O.build_variant(str(path), str(tmp_path / "libmutant.so"))
    saved = O._lib
    O._lib = mutant
    try:
        with pytest.raises(AssertionError):
            pin()
    finally:
        gc.collect()                     # oracle meshes made by the mutant are freed by it
        O._lib = saved
