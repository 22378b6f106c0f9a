"""The oracle's pins have teeth: plant a plausible mistake in a copy of the
oracle sources (on the CPU), rebuild it, and check that a pin fails.

Each mutation is a one-line edit of the kind a careful reading could miss: a
flipped dissipation sign, min instead of max in the wave speed, a wrong
Jacobian entry, a wrong lifting factor, a dropped pressure term, a wrong Pade
coefficient, a broken augmented shift or scaling, a wrong stepper
coefficient, a wrong quadrature weight, a wrong entropy-flux coefficient, a
flipped LDG switch, a wrong Dirichlet trace, and in the entropy viscosity a
dropped half on the mean divergence, h instead of h^2, a missing 1/h on the
face jump and a wrong element size, and a loose acceptance in the cost-based
Krylov adaptivity, a slip mirror or a diffusive flux through a wall, and half
the face-dependent entropy-flux penalty.
"""
import os
import shutil

import pytest

import oracle
from tests import test_oracle_adapt as ad
from tests import test_oracle_dg as dg
from tests import test_oracle_euler3d as e3
from tests import test_oracle_ev as ev
from tests import test_oracle_iop as iop
from tests import test_oracle_phi as phi
from tests import test_oracle_refelem as refelem
from tests import test_oracle_shock as sh
from tests import test_oracle_steppers as steppers
from tests import test_oracle_viscous as viscous
from tests import test_oracle_walls as wl

MUTATIONS = {
    "dissipation_sign": ("dg.cpp", "0.5 * lam * (um[c] - up[c])", "0.5 * lam * (up[c] - um[c])",
                         lambda: dg.test_burgers_upwind_energy(0.9, 1)),
    "lambda_min": ("dg.cpp", "std::fmax(wave_speed(g, qm, dir), wave_speed(g, qp, dir))",
                   "std::fmin(wave_speed(g, qm, dir), wave_speed(g, qp, dir))",
                   lambda: dg.test_piecewise_constant_rusanov(1)),
    "jacobian_entry": ("dg.cpp", "acc += gt * n[a] * v[iE];", "acc += gm * n[a] * v[iE];",
                       lambda: dg.test_jvp_equals_complex_step(2)),
    "lift_factor": ("dg.cpp", "res[c] -= (2.0 / h[dir]) / g.w[a] * (fstar_n - f_n);",
                    "res[c] -= (2.0 / h[dir]) * g.w[a] * (fstar_n - f_n);",
                    lambda: dg.test_piecewise_constant_rusanov(3)),
    "energy_flux": ("dg.cpp", "f[iE] = (q[iE] + p) * un;", "f[iE] = q[iE] * un;",
                    lambda: steppers.test_vortex_spatial_order(2)),
    "pade_coeff": ("expm.cpp", "(k * (2 * q - k + 1))", "(k * (2 * q - k))",
                   lambda: phi.test_expm_vs_scipy(12, 1.0)),
    "augmented_shift": ("krylov.cpp", "y[n + k] = x[n + k + 1];", "y[n + k + 1] = x[n + k];",
                        lambda: phi.test_krylov_dense_random(3)),
    "eta_scaling": ("krylov.cpp", "z[n + p - 1] = 1.0 / eta;", "z[n + p - 1] = eta;",
                    lambda: phi.test_krylov_dense_random(2)),
    "epi3_coeff": ("steppers.cpp", "(2.0 / 3.0) * (Rp[i]", "0.5 * (Rp[i]",
                   lambda: steppers.test_temporal_order_burgers("epi3", 3.0)),
    "exprb32_coeff": ("steppers.cpp", "b3[i] = 2.0 * (R2[i]", "b3[i] = 1.0 * (R2[i]",
                      lambda: steppers.test_temporal_order_burgers("exprb32", 3.0)),
    "ef_coeff": ("dg.cpp", "up[0] * up[0]) /", "up[0] * up[0] * 2.0) /",
                 lambda: viscous.test_entropy_flux_piecewise_constant(0.0)),
    "ldg_qstar_sign": ("dg.cpp", "qstar = 0.5 * (qL + qR) + g.beta * (qL - qR);",
                       "qstar = 0.5 * (qL + qR) - g.beta * (qL - qR);",
                       lambda: viscous.test_diffusion_energy_identity(0.5, oracle.BC_PERIODIC, 2)),
    "dirichlet_ustar": ("dg.cpp", "T ustar = T(0.0);  // Dirichlet end: u** = 0",
                        "T ustar = u[(size_t)e * n1 + i];",
                        lambda: viscous.test_diffusion_energy_identity(0.0, oracle.BC_DIRICHLET, 2)),
    "normal_speed": ("dg.cpp", "return std::fabs(u[dir]) + a;", "return std::fabs(u[0]) + a;",
                     lambda: e3.test_axis_permutation(1)),
    "ev_face_flux": ("dg.cpp", "(0.5 * (fm + fp) - fm)", "(0.5 * (fm - fp) - fm)",
                     lambda: ev.test_diffusion_symmetric_negative(3)),
    "ev_half_divergence": ("dg.cpp", "0.5 * (div[0] + div[1])", "(div[0] + div[1])",
                           lambda: ev.test_nu_E_polynomial_entropy_closed_form()),
    "ev_h_squared": ("dg.cpp", "g.ev_ce * he * he * std::fmax(rmax, jmax / he)",
                     "g.ev_ce * he * std::fmax(rmax, jmax / he)",
                     lambda: ev.test_nu_E_smooth_state_with_element_jumps(0.05, 1e9)),
    "ev_jump_over_h": ("dg.cpp", "g.ev_ce * he * he * std::fmax(rmax, jmax / he)",
                       "g.ev_ce * he * he * std::fmax(rmax, jmax)",
                       lambda: ev.test_nu_E_polynomial_entropy_closed_form()),
    "ev_h_circumradius": ("dg.cpp", "std::sqrt(g.hx * g.hx + g.hy * g.hy) / p",
                          "std::fmax(g.hx, g.hy) / p",
                          lambda: ev.test_nu_E_smooth_state_with_element_jumps(0.05, 1e9)),
    "adapt_acceptance": ("krylov.cpp", "const bool ok = om <= 1.0;", "const bool ok = om <= 1e4;",
                         lambda: ad.test_adapt_accuracy_and_checks("burgers", 30.0, 2, 0)),
    "wall_slip_mirror": ("dg.cpp", "    out[1] = -q[1];", "    out[1] = q[1];",
                         lambda: wl.test_constant_state_wall_flux_is_textbook_rusanov()),
    "wall_diffusive_flux": ("dg.cpp", "(double)s * (0.0 - fm);", "(double)s * (fm - fm);",
                            lambda: wl.test_diffusion_with_walls_symmetric_negative(3)),
    "ef_local_penalty": ("dg.cpp", "2.0 * g.kappa / (100.0 * g.hx) + lam",
                         "2.0 * g.kappa / (100.0 * g.hx) + 0.5 * lam",
                         lambda: sh.test_local_penalty_piecewise_constant(0.0)),
    "iop_window": ("krylov.cpp", "std::max(0, j - iop)", "std::max(0, j - iop - 1)",
                   lambda: iop.test_arnoldi_relation_and_band(2)),
    "lgl_weight": ("refelem.cpp", "w[i] = 2.0 / (p * (p + 1.0) * P * P);",
                   "w[i] = 2.0 / ((p + 1.0) * (p + 1.0) * P * P);",
                   lambda: refelem.test_quadrature_exactness(3)),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pin_catches_mutation(name, tmp_path):
    fname, old, new, pin = MUTATIONS[name]
    src = tmp_path / "src"
    src.mkdir()
    for f in oracle.SOURCES + ["oracle.h"]:
        shutil.copy(os.path.join(oracle.HERE, f), src / f)
    text = (src / fname).read_text()
    assert text.count(old) == 1, f"mutation anchor not unique in {fname}: {old}"
    (src / fname).write_text(text.replace(old, new))
    lib = oracle.build_at(str(src), str(tmp_path / "libmut.so"))
    pin()  # the unmutated oracle passes the pin
    with oracle.use_library(lib):
        with pytest.raises(AssertionError):
            pin()
