"""Mutation check of the oracle's pins (CPU only).

Each mutant plants one plausible mistake (a dropped term, a wrong sign, index
or factor, a transposed operand) in a private copy of lbm_oracle.c, builds it
under a temporary name and runs the pins against it.  Every mutant must make
at least one pin fail; the real oracle source is never modified.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle_pins as P
from oracle import build as B
from oracle import oracle as O

SRC = os.path.join(os.path.dirname(B.__file__), "lbm_oracle.c")

# (name, text in lbm_oracle.c, replacement)
MUTANTS = [
    ("feq_drop_quadratic", "+ 0.5 * eu * eu / (CS2 * CS2) - 0.5 * uu / CS2));",
     "- 0.5 * uu / CS2));"),
    ("feq_mu_factor", "out[i] = L->w[i] * (gamma * mu / CS2 +", "out[i] = L->w[i] * (gamma * mu +"),
    ("omega_sign", "return L->w[i] * (1.0 + eu / CS2 +", "return L->w[i] * (1.0 - eu / CS2 +"),
    ("geq_cs2", "out[i] = L->w[i] * p + CS2 * rho * (omega(L, i, u) - L->w[i]);",
     "out[i] = L->w[i] * p + rho * (omega(L, i, u) - L->w[i]);"),
    ("source_e_plus_u", "s += (L->e[i][k] - u[k]) * kk;", "s += (L->e[i][k] + u[k]) * kk;"),
    ("source_gradpsi_sign", "double kk = force[k] * om - (om - L->w[i]) * gpsi[k];",
     "double kk = force[k] * om + (om - L->w[i]) * gpsi[k];"),
    ("recover_full_force", "u[k] = (m1[k] / CS2 + 0.5 * fsg[k]) / denom;",
     "u[k] = (m1[k] / CS2 + fsg[k]) / denom;"),
    ("recover_denominator_sign", "double denom = rho - 0.5 * c;", "double denom = rho + 0.5 * c;"),
    ("recover_correction_sign", "force[k] = fsg[k] + c * u[k];", "force[k] = fsg[k] - c * u[k];"),
    ("pressure_sign", "*p = m0 + 0.5 * CS2 * dot(u, gradrho, L->dim);",
     "*p = m0 - 0.5 * CS2 * dot(u, gradrho, L->dim);"),
    ("grad_no_cs2", "grad[a * n + idx] = gsum[a] / CS2;", "grad[a * n + idx] = gsum[a];"),
    ("grad_transposed", "gsum[a] += L->w[i] * L->e[i][a] * v;",
     "gsum[a] += L->w[i] * L->e[i][(a + 1) % L->dim] * v;"),
    ("lap_factor", "if (lap) lap[idx] = 2.0 * lsum / CS2;", "if (lap) lap[idx] = lsum / CS2;"),
    ("mirror_off_by_one", "if (c < 0) return -c - 1;", "if (c < 0) return -c;"),
    ("dtheta_factor", "return 2.0 * p->beta * phi * (phi - 1.0) * (2.0 * phi - 1.0);",
     "return 2.0 * p->beta * phi * (phi - 1.0) * (phi - 1.0);"),
    ("dtheta_sym_sign", "return 4.0 * p->beta * phi * (phi * phi - p->phi_star * p->phi_star);",
     "return 4.0 * p->beta * phi * (phi * phi + p->phi_star * p->phi_star);"),
    ("rho_sym_offset", "return p->rho_g + (phi + p->phi_star) / (2.0 * p->phi_star) * (p->rho_l - p->rho_g);",
     "return p->rho_g + (phi + p->phi_star) / p->phi_star * (p->rho_l - p->rho_g);"),
    ("beta_kappa_sym_power", "*beta = 3.0 * sigma / (4.0 * width * p2 * p2);",
     "*beta = 3.0 * sigma / (4.0 * width * p2);"),
    ("mu_kappa_sign", "s->mu[idx] = dtheta_well(p, s->phi[idx]) - p->kappa * s->lphi[idx];",
     "s->mu[idx] = dtheta_well(p, s->phi[idx]) + p->kappa * s->lphi[idx];"),
    ("beta_kappa_swap", "*beta = 12.0 * sigma / width;", "*beta = 8.0 * sigma / width;"),
    ("gamma_no_half", "s->gamma = prm->theta_m / (prm->tau_f - 0.5);",
     "s->gamma = prm->theta_m / prm->tau_f;"),
    ("gravity_sign", "fsg[vert] += -(s->rho[idx] - p->rho_ref) * p->gravity;",
     "fsg[vert] += (s->rho[idx] - p->rho_ref) * p->gravity;"),
    ("surface_force_dropped", "fsg[k] = s->mu[idx] * s->gphi[k * n + idx];",
     "fsg[k] = 0.0 * s->gphi[k * n + idx];"),
    ("correction_sign", "double c = sw * s->drho_dphi * p->theta_m * s->lmu[idx];",
     "double c = -sw * s->drho_dphi * p->theta_m * s->lmu[idx];"),
    ("correction_uses_lap_phi", "double c = sw * s->drho_dphi * p->theta_m * s->lmu[idx];",
     "double c = sw * s->drho_dphi * p->theta_m * s->lphi[idx];"),
    ("gradpsi_sign", "s->gpsi[k * n + idx] -= CS2 * s->drho_dphi * s->gphi[k * n + idx];",
     "s->gpsi[k * n + idx] += CS2 * s->drho_dphi * s->gphi[k * n + idx];"),
    ("tau_no_half", "s->tau[idx] = 0.5 + nu / CS2;", "s->tau[idx] = nu / CS2;"),
    ("mu_gas_inverted", "s->mu_g = s->mu_l / prm->mu_ratio;", "s->mu_g = s->mu_l * prm->mu_ratio;"),
    ("density_closure", "return p->rho_g + phi * (p->rho_l - p->rho_g);",
     "return p->rho_l + phi * (p->rho_l - p->rho_g);"),
    ("collide_f_sign", "s->f[i * n + idx] = fi - (fi - fe[i]) / tf;",
     "s->f[i * n + idx] = fi + (fi - fe[i]) / tf;"),
    ("collide_g_no_trapezoid", "+ (1.0 - 1.0 / (2.0 * tg)) * src[i];", "+ src[i];"),
    ("stream_push", "s[a] = c[a] - L->e[i][a];", "s[a] = c[a] + L->e[i][a];"),
    ("bounce_back_same_dir", "int j = bb ? L->opp[i] : i;", "int j = i;"),
    ("diag_weight", "double w = 2.0 * (ph - s->phi_g) / (s->phi_l - s->phi_g) - 0.5;",
     "double w = 2.0 * (ph - s->phi_g) / (s->phi_l - s->phi_g) - 1.0;"),
    ("leelin_thermo_sign", "ph * dtheta_well(prm, ph) - theta_well(prm, ph);",
     "ph * dtheta_well(prm, ph) + theta_well(prm, ph);"),
    ("leelin_no_grad_lambda", "div += gl[a * n + idx] * gq[a * n + idx];",
     "div += 0.0 * gl[a * n + idx] * gq[a * n + idx];"),
    ("leelin_lambda_liquid_rho", "lam[idx] = mud / (rho_of(prm, ph) * CS2);",
     "lam[idx] = mud / (prm->rho_l * CS2);"),
    ("leelin_visc_reversed", "const double mud = mu_g + (ph - phi_g) / (phi_l - phi_g) * (mu_l - mu_g);",
     "const double mud = mu_g + (phi_l - ph) / (phi_l - phi_g) * (mu_l - mu_g);"),
    ("theta_asym_power", "return p->beta * phi * phi * (phi - 1.0) * (phi - 1.0);",
     "return p->beta * phi * phi * (phi - 1.0);"),
    ("data_rate_no_time_term",
     "s->dmass[idx] = s->drho_dphi * (s->phi[idx] - s->phi_prev[idx]);",
     "s->dmass[idx] = 0.0 * s->drho_dphi * (s->phi[idx] - s->phi_prev[idx]);"),
    ("data_rate_phi_prev_frozen", "memcpy(s->phi_prev, s->phi, (size_t)s->n * sizeof(double));",
     ";"),
    ("data_rate_corrected_u", "for (int k = 0; k < dim; ++k) s->rhou[k * n + idx] = s->rho[idx] * uu[k];",
     "for (int k = 0; k < dim; ++k) s->rhou[k * n + idx] = s->rho[idx] * s->u[k * n + idx];"),
    ("data_rate_sign", "if (p->remove_fa == 2) c = s->dmass[idx];",
     "if (p->remove_fa == 2) c = -s->dmass[idx];"),
    ("d3q19_edge_weight", "L->w[i] = (i == 0) ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);",
     "L->w[i] = (i == 0) ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 18.0);"),
    ("d3q19_edge_vector", "{-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},",
     "{-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, 1}, {-1, 0, -1},"),
]

FAST_CHECKS = [c for c in P.ALL_CHECKS]


def _build_mutant(tmp, name, old, new):
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutant {name}: anchor not unique/missing"
    src = os.path.join(tmp, f"{name}.c")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    shutil.copy(os.path.join(os.path.dirname(SRC), "lbm_oracle.h"), tmp)
    out = os.path.join(tmp, f"lib{name}.so")
    subprocess.run(["gcc", "-std=c99", "-O1", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-w", src, "-o", out, "-lm"], check=True)
    return out


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    with tempfile.TemporaryDirectory() as tmp:
        lib = O.load(_build_mutant(tmp, name, old, new))
        failed = []
        for chk in FAST_CHECKS + [P.check_flat_interface]:
            try:
                chk(lib)
            except (AssertionError, ValueError, FloatingPointError):
                failed.append(chk.__name__)
                break
        assert failed, f"no pin catches mutant {name}"
