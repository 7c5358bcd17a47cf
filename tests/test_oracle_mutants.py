"""The oracle's pins reject plausible mistakes.

Each case plants one mistake in a copy of the oracle source (on the CPU),
builds it, and runs the pin suite against it; the suite must fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "eik_oracle.c")

MUTANTS = {
    "two_sided_operand": ("0.5 * (a + b + sqrt(", "0.5 * (a + a + sqrt("),
    "one_sided_step": ("return lo + delta;", "return lo + 0.5 * delta;"),
    "dropped_factor_2": ("sqrt(2.0 * delta * delta - d * d)", "sqrt(delta * delta - d * d)"),
    "max_for_min": ("double b = uS < uN ? uS : uN;", "double b = uS > uN ? uS : uN;"),
    "branch_sign": ("if (fabs(d) >= delta)", "if (d >= delta)"),
    "fmsm_upwind_index": ("nb(g, V, i, j - sy)", "nb(g, V, i, j + sy)"),
    "fmsm_dir_swap": ("if (W) d |= (1 << 0) | (1 << 1);", "if (W) d |= (1 << 0) | (1 << 2);"),
    "add_criterion_sign": ("V[ki] < V[kj]) add = 1;", "V[ki] > V[kj]) add = 1;"),
    "fmm_skip_decrease_key": ("      } else {\n        heap_up(&H, H.pos[kk]);\n      }\n    }\n  }\n  if (nacc)",
                              "      }\n    }\n  }\n  if (nacc)"),
    "source_first_removal": ("(first && g.src[ki])", "(0 && g.src[ki])"),
}

# Mistakes in the 3-D FMSM (checked against the 3-D pins)
MUTANTS3 = {
    "fmsm3_upwind_z": ("nb3(g, V, i, j, k - sz), g->delta[x])", "nb3(g, V, i, j, k + sz), g->delta[x])"),
    "fmsm3_direction_swap": ("allow[a] = (lo ? 1 : 0) | (hi ? 2 : 0);", "allow[a] = (lo ? 2 : 0) | (hi ? 1 : 0);"),
    "fmsm3_centre_z": ("int ks[2] = {(lo[2] + hi[2] - 1) / 2, (lo[2] + hi[2]) / 2};",
                       "int ks[2] = {lo[2], lo[2]};"),
    "fmsm3_thin_axis_doubled": ("if ((thin_axes >> a) & 1) allow[a] = 1;", "if (0) allow[a] = 1;"),
    "fmsm3_source_cells_one_sweep": ("        } while (ch);\n        S.sweeps += sw;\n      } else {\n        int ci[3]",
                                     "        } while (0);\n        S.sweeps += sw;\n      } else {\n        int ci[3]"),
}


def run_pins_against(old, new, tmp_path, test_file):
    text = open(SRC).read()
    assert text.count(old) >= 1, "mutation site not found"
    mutated = text.replace(old, new, 1)
    c = tmp_path / "eik_oracle.c"
    c.write_text(mutated)
    (tmp_path / "eik_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "eik_oracle.h")).read())
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                    "-o", str(so), str(c), "-lm"], check=True)
    env = dict(os.environ, EIK_ORACLE_LIB=str(so))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", test_file)],
                          env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    r = run_pins_against(*MUTANTS[name], tmp_path, "test_oracle.py")
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS3))
def test_3d_pins_reject_mutant(name, tmp_path):
    r = run_pins_against(*MUTANTS3[name], tmp_path, "test_oracle3d.py")
    assert r.returncode != 0, f"mutant {name} passed every 3-D pin:\n{r.stdout[-2000:]}"
