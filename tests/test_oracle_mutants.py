"""The event-law pins fail on plausible mistakes in the oracle (CPU only).

Each case copies the oracle source, plants one mistake in the copy, builds
it in a temporary directory and runs the event-law pins against that build
in a process of its own (``SGPM_ORACLE_LIB``).  The pins must fail.  The
mistakes are the ones a reading of Sec. 3 (eq. dt, eq. gamma_tot, eq. update)
and Sec. 4.1 (eq. deltat) could plausibly make:

* the mechanism intervals normalised by the node's own total rate S_q
  instead of the majorant G = (1 + alpha) max_q S_q;
* the free flight drawn with max_q S_q, i.e. without the self-scattering
  factor (1 + alpha);
* the optical emission and absorption final states swapped;
* the optical Bose factors (n + 1 for emission, n for absorption) swapped.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sgpm_oracle.c")

MUTANTS = {
    "selection_by_node_rate": [
        ("if (su < cum / G) { ell = m + 1; break; }",
         "if (su < cum / S[q]) { ell = m + 1; break; }")],
    "free_flight_without_self_scattering": [
        ("double dtc = -log(xi) / G;", "double dtc = -log(xi) / Smax;")],
    "optical_final_states_swapped": [
        ("final_magnitude(s, kx, ky, e0, -s->hw_O)", "final_magnitude(s, kx, ky, e0, +s->HWTMP)"),
        ("final_magnitude(s, kx, ky, e0, +s->hw_O)", "final_magnitude(s, kx, ky, e0, -s->hw_O)"),
        ("+s->HWTMP", "+s->hw_O")],
    "optical_bose_factors_swapped": [
        ("sc[1] * s->C_O * (s->n_O + 1.0) * eOm", "sc[1] * s->C_O * s->n_O * eOm"),
        ("sc[2] * s->C_O * s->n_O * eOp", "sc[2] * s->C_O * (s->n_O + 1.0) * eOp")],
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_event_law_pins_catch_the_mutant(tmp_path, name):
    src = open(SRC).read()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    shutil.copy(os.path.join(ROOT, "oracle", "sgpm_oracle.h"), tmp_path)
    csrc = tmp_path / "sgpm_oracle.c"
    csrc.write_text(src)
    so = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(so), str(csrc), "-lm"], check=True, cwd=tmp_path)
    env = dict(os.environ, SGPM_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_event_law.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert "failed" in r.stdout and r.returncode != 0, r.stdout[-2000:]
