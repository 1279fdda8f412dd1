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
from tests import test_oracle_hex as T_hex
from tests import test_oracle_viscous as T_visc

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
    # the viscosity law with the temperature ratio inverted
    "mu_law": ("pow((p0 / s0.rho) / p->T_ref, p->mu_exp)",
               "pow(p->T_ref / (p0 / s0.rho), p->mu_exp)",
               T_visc.test_shear_stress_is_navier_stokes_with_the_power_law_viscosity),
    # the Prandtl correction with the factor reversed
    "prandtl_factor": ("Fl[4] += (1.0 / p->prandtl - 1.0) * qh;",
                       "Fl[4] += (1.0 - 1.0 / p->prandtl) * qh;",
                       lambda: T_visc.test_heat_flux_is_fourier_with_the_prandtl_number(0.72, (0.0, 0.0, 0.0))),
    # the heat flux measured without the frame velocity's momentum term
    "prandtl_frame": ("const double qh = Fl[4] - (U0[0] * Fl[1] + U0[1] * Fl[2] + U0[2] * Fl[3]) + u2 * Fl[0]",
                      "const double qh = Fl[4] + u2 * Fl[0]",
                      lambda: T_visc.test_heat_flux_is_fourier_with_the_prandtl_number(0.72, (0.3, 0.2, 0.0))),
    # the far field's incoming invariant with the wrong sign of the sound-speed term
    "farfield_rminus": ("Rm = vf - 2.0 * cf / (g - 1.0);", "Rm = vf + 2.0 * cf / (g - 1.0);",
                        lambda: T_visc.test_farfield_state_by_its_invariants(0.3)),
    # the far field's entropy always from the interior
    "farfield_entropy": ("const double ent = outflow ? si.p / pow(si.rho, g) : pf / pow(rf, g);",
                         "const double ent = si.p / pow(si.rho, g);",
                         lambda: T_visc.test_farfield_state_by_its_invariants(-0.3)),
    # the wall ghost negating only the normal momentum (a slip wall)
    "wall_slip": ("out[0] = q[0]; out[1] = -q[1]; out[2] = -q[2]; out[3] = -q[3]; out[4] = q[4];",
                  "out[0] = q[0]; out[1] = -q[1]; out[2] = q[2]; out[3] = q[3]; out[4] = q[4];",
                  T_visc.test_wall_ghost_and_wall_flux),
    # a hex sub-stencil with the wrong side face
    "hex_substencil": ("{0,1,2},{0,2,3},{0,3,4},{0,4,1},{5,1,2}", "{0,1,2},{0,2,3},{0,3,4},{0,4,2},{5,1,2}",
                       T_hex.test_hex_stencils_follow_the_lattice),
    # the bilinear face's Gauss weight without the 1/4 of the 2x2 rule on [0, 1]^2
    "hex_face_weight": ("gw[g] = 0.25 * len;", "gw[g] = 0.5 * len;",
                        T_hex.test_bilinear_face_points_give_the_exact_vector_area_and_closure),
    # the hex cell rule with the middle Gauss weight of the 2-point rule
    "hex_cell_rule": ("GL3W[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0}", "GL3W[3] = {5.0 / 18.0, 9.0 / 18.0, 5.0 / 18.0}",
                      T_hex.test_affine_hex_volume_centroid_and_moments),
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
