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
