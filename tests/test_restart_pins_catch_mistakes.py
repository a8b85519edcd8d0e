"""The restart pins (tests/test_oracle_restart.py) fail on plausible mistakes in the oracle's
restart driver.

Each case plants one mistake in a copy of qcqp_oracle.c (CPU only, in a temporary directory),
builds that copy with the oracle's own flags and runs the restart pins against it in a child
process (ORACLE_LIB names the copy).  The run must report failures.  The mistakes:
  * the adaptive test of eq. (ada_restart) never fires;
  * a successful adaptive test leaves the reference G_xi where it was;
  * a restart keeps the ending epoch's tau and tau_{-1} instead of re-entering the first line of
    Algorithm 1 (Algorithm 2, §4.1);
  * a restart keeps the ending epoch's gamma;
  * the restart point is the last iterate although the weighted average of Algorithm 2 is
    requested;
  * the fixed restart period K-hat is off by one.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "qcqp_oracle.c")

MISTAKES = {
    "adaptive_never_fires": (
        "if (g4[0] <= o->q_restart * Gref) { do_restart = 1; Gref = g4[0]; }",
        "if (0 && g4[0] <= o->q_restart * Gref) { do_restart = 1; Gref = g4[0]; }"),
    "reference_gap_not_reset": (
        "if (g4[0] <= o->q_restart * Gref) { do_restart = 1; Gref = g4[0]; }",
        "if (g4[0] <= o->q_restart * Gref) { do_restart = 1; }"),
    "restart_keeps_tau": (
        "            restart_point(&S);\n            epoch_init(&S, &ep);",
        "            restart_point(&S);\n            { double kt = ep.tau, kp = ep.tau_prev; "
        "epoch_init(&S, &ep); ep.tau = kt; ep.tau_prev = kp; }"),
    "restart_keeps_gamma": (
        "            restart_point(&S);\n            epoch_init(&S, &ep);",
        "            restart_point(&S);\n            { double kg = ep.gam; epoch_init(&S, &ep); ep.gam = kg; }"),
    "restart_from_last_iterate": (
        "    if (S->o->restart_from_average && S->T > 0.0) {",
        "    if (0 && S->o->restart_from_average && S->T > 0.0) {"),
    "fixed_period_off_by_one": (
        "if (o->restart == 1 && ep.ke >= o->restart_every) do_restart = 1;",
        "if (o->restart == 1 && ep.ke > o->restart_every) do_restart = 1;"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_restart_pins_fail_on_planted_mistake(name, tmp_path):
    from oracle import build
    src = open(SRC).read()
    old, new = MISTAKES[name]
    assert src.count(old) == 1, f"the text the mistake replaces is no longer in qcqp_oracle.c: {old!r}"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = build.build_from(str(path), str(tmp_path / f"lib_{name}.so"))
    env = dict(os.environ, ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join("tests", "test_oracle_restart.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 1 and " failed" in r.stdout, tail
