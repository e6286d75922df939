"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle source (on the CPU, in a
temporary directory), builds it, and runs the pin suite against the copy; the
suite must fail.  The real oracle is untouched.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "stratego_oracle.c")

# (name, original text, planted mistake, pin tests expected to notice)
MUTANTS = [
    ("spy beats marshal when defending too",
     "if (a == SPY && d == MARSHAL) return BATTLE_ATTACKER;",
     "if (a == SPY && d == MARSHAL) return BATTLE_ATTACKER;\n    if (a == MARSHAL && d == SPY) return BATTLE_DEFENDER;",
     "battle_table"),
    ("scouts jump over pieces",
     "                if (o != EMPTY) break;\n",
     "                if (o != EMPTY) continue;\n",
     "brute_force"),
    ("lakes are passable",
     "                if (is_lake(y)) break;\n                int o = st->board[y];",
     "                int o = st->board[y];\n                if (o == LAKE) o = EMPTY;",
     "brute_force"),
    ("probabilities rounded down",
     "return (int)((510 * num + den) / (2 * den));",
     "return (int)((255 * num) / den);",
     "probability"),
    ("moved pieces may be bombs",
     "        if (!is_movable_type(t)) { *num = 0; *den = 1; return; }\n        *num = hs->n[t];\n        *den = movable_slots;",
     "        *num = hs->n[t];\n        *den = hs->H;",
     "probability"),
    ("blue's view not rotated",
     "static int frame(int o, int sq) { return o == 0 ? sq : 99 - sq; }",
     "static int frame(int o, int sq) { (void)o; return sq; }",
     "probability_channels_at_ply0 or brute_force_enumeration"),
    ("wrong Philox multiplier",
     "uint64_t p0 = (uint64_t)0xD2511F53u * c[0];",
     "uint64_t p0 = (uint64_t)0xD2511F55u * c[0];",
     "philox"),
    ("tie reported as a loss for the attacker",
     "px->death_cause = !rY ? 3 : 2;",
     "px->death_cause = !rY ? 3 : 1;",
     "battle_deaths"),
    ("threat on a revealed bomb recorded",
     "            if (Y->revealed && !is_movable_type(Y->type)) continue;\n            st->piece[X].threat",
     "            st->piece[X].threat",
     "threat"),
    ("an attack counts as an evasion",
     "if (A >= 0 && adjacent(from, a) && target == EMPTY && !adjacent(to, a) &&",
     "if (A >= 0 && adjacent(from, a) && !adjacent(to, a) &&",
     "evasion"),
    ("k-move rule off by one",
     "if (st->battleless >= cfg->k_battleless) {",
     "if (st->battleless > cfg->k_battleless) {",
     "terminal"),
    ("two-square spans that only touch count as shared",
     "    return lo < hi;\n}",
     "    return lo <= hi;\n}",
     "two_square"),
    ("magnet counts the destination square's moves",
     "out[k++] = 1.0f / (float)(P * moves_from(m, a / 100));",
     "out[k++] = 1.0f / (float)(P * moves_from(m, a % 100));",
     "magnet"),
    ("magnet sampler never picks the last piece",
     "int r1 = (int)bounded(w[1], (uint32_t)P);",
     "int r1 = (int)bounded(w[1], (uint32_t)(P > 1 ? P - 1 : 1));",
     "magnet_sampler"),
    ("search policy pushes away from the magnet",
     "e[k] = ((double)q[j] + alpha * log(rho) + beta * (double)logpi[j]) / (alpha + beta);",
     "e[k] = ((double)q[j] - alpha * log(rho) + beta * (double)logpi[j]) / (alpha + beta);",
     "search_policy"),
    ("chasing rule ignores the returning exception",
     "    if (st->ring_to[prev] == from && st->ring_from[prev] == to) return 0;\n",
     "",
     "chas"),
    ("chasing rule skips the chase's first position",
     "    for (int k = 1; k <= K; k++) {                             /* positions P_{L-1}, ..., P_{L-K} */",
     "    for (int k = 1; k < K; k++) {                             /* positions P_{L-1}, ..., P_{L-K} */",
     "chas"),
    ("setup shuffle skips the last swap",
     "for (int i = 39; i >= 1; i--) {\n        int j = (int)bounded(stream_next(&ws), (uint32_t)(i + 1));",
     "for (int i = 39; i >= 2; i--) {\n        int j = (int)bounded(stream_next(&ws), (uint32_t)(i + 1));",
     "setup or initial_legal"),
]


@pytest.mark.parametrize("name,orig,bad,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, orig, bad, pins):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation anchor not found once: {name}"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(orig, bad))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-shared", "-fPIC", str(mutant),
                           "-o", str(lib), "-lm"])
    env = dict(os.environ, STRATEGO_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    kexpr = " or ".join(f"{w}" for w in pins.split(" or "))
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-x", "-q", "-p", "no:cacheprovider", "-k", kexpr],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert "passed" in r.stdout or "failed" in r.stdout, r.stdout + r.stderr
    assert r.returncode != 0, f"planted mistake survived the pins: {name}\n{r.stdout[-2000:]}"
