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

# (name, original text, planted mistake, pin tests expected to notice: a -k
# expression over tests/test_oracle_pins.py, or "file.py::expression")
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
    ("chasing rule compares positions with the other side to move",
     "if ((k & 1) && memcmp(b, after, sizeof(b)) == 0) return 1;",
     "if (memcmp(b, after, sizeof(b)) == 0) return 1;",
     "chas"),
    ("chasing rule looks back over 30 plies only",
     "    int K = L < st->ring_count ? L : st->ring_count;           /* ring_count <= CHASE_WINDOW */",
     "    int K = L < st->ring_count ? L : st->ring_count;\n    if (K > 30) K = 30;",
     "chas"),
    ("setup shuffle skips the last swap",
     "for (int i = 39; i >= 1; i--) {\n        int j = (int)bounded(stream_next(&ws), (uint32_t)(i + 1));",
     "for (int i = 39; i >= 2; i--) {\n        int j = (int)bounded(stream_next(&ws), (uint32_t)(i + 1));",
     "setup or initial_legal"),
    # channel placement (App. C.1 channel tables, App. C.2 move planes)
    ("own types written to channel 11 - t",
     "put(out, P->type, f, 1);",
     "put(out, 11 - P->type, f, 1);",
     "test_oracle_channels.py::own_type"),
    ("evasion and adjacency groups swapped",
     "if (P->evade & (1u << j)) put(out, hbase + 11 + j, f, 1);\n"
     "            if (P->adj & (1u << j)) put(out, hbase + 22 + j, f, 1);",
     "if (P->evade & (1u << j)) put(out, hbase + 22 + j, f, 1);\n"
     "            if (P->adj & (1u << j)) put(out, hbase + 11 + j, f, 1);",
     "test_oracle_channels.py::threat_evasion"),
    ("death-cause offset 10 (c mod 6)",
     "10 * (P->death_cause - 1)",
     "10 * (P->death_cause % 6)",
     "test_oracle_channels.py::causes_of_death"),
    ("move planes oldest first",
     "int slot = (st->ply - 1 - i) & (RING - 1);",
     "int slot = (st->ply - st->ring_count + i) & (RING - 1);",
     "test_oracle_channels.py::recent_moves"),
    ("opponent threat group starts at 77",
     "int hbase = own ? 43 : 76;",
     "int hbase = own ? 43 : 77;",
     "test_oracle_channels.py::threat_evasion"),
    ("start-square channel not in the observer's frame",
     "put(out, 355 + frame(o, start_square(id)), f, 1);",
     "put(out, 355 + start_square(id), f, 1);",
     "test_oracle_channels.py::start_square"),
    ("captured pieces marked at their death square",
     "put(out, (own ? 109 : 120) + slot11, frame(o, start_square(id)), 1);",
     "put(out, (own ? 109 : 120) + slot11, frame(o, P->death_square), 1);",
     "test_oracle_channels.py::captured"),
    ("protected-against and been-protected-by groups swapped",
     "if (P->prot_against & (1u << j)) put(out, gbase + 13 + j, f, 1);\n"
     "            if (P->been_by & (1u << j)) put(out, gbase + 26 + j, f, 1);",
     "if (P->prot_against & (1u << j)) put(out, gbase + 26 + j, f, 1);\n"
     "            if (P->been_by & (1u << j)) put(out, gbase + 13 + j, f, 1);",
     "test_oracle_channels.py::protection"),
    ("own moved pieces on the opponent's moved channel",
     "if (P->moved) put(out, 39, f, 1);",
     "if (P->moved) put(out, 40, f, 1);",
     "test_oracle_channels.py::hidden_empty_moved"),
    ("k-move fraction on channel 41",
     "put(out, 41, f, (uint8_t)v41);\n        put(out, 42, f, (uint8_t)v42);",
     "put(out, 41, f, (uint8_t)v42);\n        put(out, 42, f, (uint8_t)v41);",
     "test_oracle_channels.py::fractions"),
    ("move sources written as +1",
     "put(out, 456 + i, frame(o, st->ring_from[slot]), 0xFF);",
     "put(out, 456 + i, frame(o, st->ring_from[slot]), 0x01);",
     "test_oracle_channels.py::recent_moves"),
    ("probabilities of own pieces written to the opponent's group",
     "int pbase = own ? 24 : 12;",
     "int pbase = own ? 12 : 24;",
     "test_oracle_channels.py::probabilities"),
    # random-number conventions (recomputed from the stated conventions)
    ("uniform sampler reads word y",
     "int r = (int)bounded(w[0], (uint32_t)n);",
     "int r = (int)bounded(w[1], (uint32_t)n);",
     "test_oracle_conventions.py::uniform_move"),
    ("setup shuffled by an ascending Fisher-Yates",
     "for (int i = 39; i >= 1; i--) {\n        int j = (int)bounded(stream_next(&ws), (uint32_t)(i + 1));",
     "for (int i = 0; i < 39; i++) {\n        int j = i + (int)bounded(stream_next(&ws), (uint32_t)(40 - i));",
     "test_oracle_conventions.py::setup"),
    ("magnet sampler picks the piece with word x",
     "int r1 = (int)bounded(w[1], (uint32_t)P);",
     "int r1 = (int)bounded(w[0], (uint32_t)P);",
     "test_oracle_conventions.py::magnet"),
    ("resample shuffles the movable types by an ascending Fisher-Yates",
     "for (int i = L - 1; i >= 1; i--) {\n        int j = (int)bounded(stream_next(&ws), (uint32_t)(i + 1));",
     "for (int i = 0; i < L - 1; i++) {\n        int j = i + (int)bounded(stream_next(&ws), (uint32_t)(L - i));",
     "test_oracle_conventions.py::resample"),
    ("resample places the Bombs before the Flag",
     "assigned[unmoved[i]] = (i < hs.n[FLAG]) ? FLAG : BOMB;",
     "assigned[unmoved[i]] = (i >= I - hs.n[FLAG]) ? FLAG : BOMB;",
     "test_oracle_conventions.py::resample"),
    # known Scouts (a move of more than one square, App. A)
    ("known Scouts stay in the unknown set",
     "if (!p->alive || p->revealed || p->long_move) {",
     "if (!p->alive || p->revealed) {",
     "test_oracle_channels.py::known_scout"),
    ("long moves not recorded",
     "    if (!adjacent(from, to)) st->piece[X].long_move = 1;\n",
     "",
     "long_moves"),
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
    target, kexpr = pins.split("::") if "::" in pins else ("test_oracle_pins.py", pins)
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", target),
                        "-x", "-q", "-p", "no:cacheprovider", "-k", kexpr],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert "passed" in r.stdout or "failed" in r.stdout, r.stdout + r.stderr
    assert r.returncode != 0, f"planted mistake survived the pins: {name}\n{r.stdout[-2000:]}"
    if target == "test_oracle_channels.py":   # the failing assertion names the channel
        assert " channel " in r.stdout, r.stdout[-2000:]
