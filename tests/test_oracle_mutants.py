"""Plants plausible mistakes in a copy of the oracle (on the CPU) and checks that the pins catch them.

Each mutant rewrites one expression of pdhg_oracle.c in a temporary copy, builds it, and runs the
pins against it until one fails. A mutant that passes every pin would mean the pins leave that part
of the oracle unchecked.
"""
import os

import pytest

import oracle
import oracle_pins as P

MUTANTS = {
    # dropped extrapolation term in the dual step
    "dual_extrapolation": ("yn[i] = proj_y(y[i] + sigma * (b[i] - 2.0 * axn[i] + ax[i]), sense[i]);",
                           "yn[i] = proj_y(y[i] + sigma * (b[i] - axn[i]), sense[i]);"),
    # wrong sign of A'y in the primal step
    "primal_sign": ("xn[j] = clip(x[j] - tau * (c[j] - aty[j]), l[j], u[j]);",
                    "xn[j] = clip(x[j] - tau * (c[j] + aty[j]), l[j], u[j]);"),
    # dual sign sets of >= and <= rows swapped
    "dual_projection": ("if (s == 'G') return y > 0.0 ? y : 0.0;", "if (s == 'L') return y > 0.0 ? y : 0.0;"),
    # reduced-cost cone of a lower-bounded column flipped
    "lambda_cone": ("if (lf) return g > 0.0 ? g : 0.0;", "if (lf) return g < 0.0 ? g : 0.0;"),
    # upper-bound term of the dual objective with the wrong sign
    "dual_objective": ("bound_terms += u[j] * lam;", "bound_terms -= u[j] * lam;"),
    # bounds scaled in the wrong direction
    "bound_scaling": ("ls[j] = isfinite(lp->l[j]) ? lp->l[j] / Dc[j] : lp->l[j];",
                      "ls[j] = isfinite(lp->l[j]) ? lp->l[j] * Dc[j] : lp->l[j];"),
    # right-hand side scaled in the wrong direction
    "rhs_scaling": ("bs[i] = Dr[i] * lp->b[i];", "bs[i] = lp->b[i] / Dr[i];"),
    # column factor dropped when the matrix is rescaled
    "matrix_scaling": ("sv[k] = sv[k] / (rho[i] * kap[ci[k]]);", "sv[k] = sv[k] / rho[i];"),
    # primal residual of >= rows with the wrong sign test
    "primal_residual": ("if (sense[i] == 'G') t = t > 0.0 ? t : 0.0;", "if (sense[i] == 'G') t = t < 0.0 ? t : 0.0;"),
    # dual residual scaled back with the wrong factor
    "dual_residual_unscale": ("double rdo = Dc ? rd / Dc[j] : rd;", "double rdo = Dc ? rd * Dc[j] : rd;"),
    # transposed operand: the transposed product uses the column index as the row index
    "transpose_index": ("tci[p] = i;", "tci[p] = ci[k] % (m > 0 ? m : 1);"),
    # warm start scaled the wrong way
    "warm_start_scaling": ("cur.x[j] = clip(o->x0 ? o->x0[j] / Dc[j] : 0.0, ls[j], us[j]);",
                           "cur.x[j] = clip(o->x0 ? o->x0[j] * Dc[j] : 0.0, ls[j], us[j]);"),
    # primal weight dropped from the step-size bound
    "step_weight": ("(omega * dx2 + dy2 / omega) / denom", "(dx2 + dy2) / denom"),
    # unscaled output
    "output_unscale": ("x_out[j] = Dc[j] * cur.x[j];", "x_out[j] = cur.x[j];"),
}

# Mistakes in the scalar rules of the method (restart test, primal weight, step size, start values).
# Any such choice still converges to the same optimum, so outcome pins cannot see them: each must
# fail the named formula pin, on hand-worked numbers.
RULE_MUTANTS = {
    "restart_sufficient_beta": ("(kkt_c <= 0.2 * kkt_anchor)", "(kkt_c <= 0.02 * kkt_anchor)", "pin_restart_rule"),
    "restart_necessary_beta": ("(kkt_c <= 0.8 * kkt_anchor && kkt_c > kkt_prev)",
                               "(kkt_c <= 0.5 * kkt_anchor && kkt_c > kkt_prev)", "pin_restart_rule"),
    "restart_no_progress_sign": ("(kkt_c <= 0.8 * kkt_anchor && kkt_c > kkt_prev)",
                                 "(kkt_c <= 0.8 * kkt_anchor && kkt_c < kkt_prev)", "pin_restart_rule"),
    "restart_artificial_beta": ("0.36 * (double)k", "0.5 * (double)k", "pin_restart_rule"),
    "restart_always_current": ("int avg = kkt_avg < kkt_cur;", "int avg = 0;", "pin_restart_rule"),
    "restart_ties_to_average": ("int avg = kkt_avg < kkt_cur;", "int avg = kkt_avg <= kkt_cur;", "pin_restart_rule"),
    "omega_smoothing_theta": ("exp(0.5 * log(dy / dx) + 0.5 * log(omega))",
                              "exp(0.3 * log(dy / dx) + 0.7 * log(omega))", "pin_primal_weight"),
    "omega_inverted": ("exp(0.5 * log(dy / dx) + 0.5 * log(omega))",
                       "exp(0.5 * log(dx / dy) + 0.5 * log(omega))", "pin_primal_weight"),
    "omega_guard_either": ("if (dx > 1e-10 && dy > 1e-10)", "if (dx > 1e-10 || dy > 1e-10)", "pin_primal_weight"),
    "omega0_unscaled": ("norm2_ord(cs, n, rev), norm2_ord(bs, m, rev)",
                        "norm2_ord(lp->c, n, rev), norm2_ord(lp->b, m, rev)", "pin_initial_values"),
    "omega0_inverted": ("return norm_c_scaled / norm_b_scaled;", "return norm_b_scaled / norm_c_scaled;",
                        "pin_initial_values"),
    "eta0_factor": ("return amax > 0.0 ? 1.0 / amax : 1.0;", "return amax > 0.0 ? 2.0 / amax : 1.0;",
                    "pin_initial_values"),
    "eta_growth_exponent": ("pow(kk, -0.6)", "pow(kk, -0.3)", "pin_step_rule"),
    "eta_shrink_exponent": ("(1.0 - pow(kk, -0.3))", "(1.0 - pow(kk, -0.5))", "pin_step_rule"),
    "eta_attempt_index": ("double kk = (double)(k + 1);", "double kk = (double)k;", "pin_step_rule"),
    "accept_strict": ("return eta <= eta_bar;", "return eta < eta_bar;", "pin_step_rule"),
    "kkt_weights_swapped": ("omega * omega * rp2 + rd2 / (omega * omega)", "rp2 / (omega * omega) + omega * omega * rd2",
                            "pin_kkt_weighted"),
    "kkt_gap_dropped": ("rd2 / (omega * omega) + gap * gap)", "rd2 / (omega * omega))", "pin_kkt_weighted"),
}


@pytest.fixture(scope="module")
def source():
    with open(oracle.SRC) as f:
        return f.read()


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutation site for {name} not found exactly once"
    src = tmp_path / f"mut_{name}.c"
    src.write_text(source.replace(old, new))
    lib = str(tmp_path / f"libmut_{name}.so")
    oracle.build(openmp=False, src=str(src), out=lib)
    caught = None
    for pin in P.ALL_PINS:
        try:
            pin(lib)
        except (AssertionError, FloatingPointError, ValueError, MemoryError) as e:  # noqa: PERF203
            caught = (pin.__name__, repr(e)[:200])
            break
    assert caught is not None, f"mutant {name} passed every pin"
    os.remove(lib)


@pytest.mark.parametrize("name", sorted(RULE_MUTANTS))
def test_rule_mutant_fails_its_formula_pin(name, source, tmp_path):
    old, new, pin_name = RULE_MUTANTS[name]
    assert source.count(old) == 1, f"mutation site for {name} not found exactly once"
    src = tmp_path / f"mut_{name}.c"
    src.write_text(source.replace(old, new))
    lib = str(tmp_path / f"libmut_{name}.so")
    oracle.build(openmp=False, src=str(src), out=lib)
    pin = getattr(P, pin_name)
    with pytest.raises(AssertionError):
        pin(lib)
    os.remove(lib)
