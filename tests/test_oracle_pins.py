"""Pins of the CPU oracle to what the paper and mathematics fix (no GPU).

Each test ties one part of the oracle to something other than its own code:
the paper's piece table, brute force over all (from, to) pairs, closed forms
at the initial position, exhaustive enumeration of hidden-type assignments,
published Philox known-answer vectors, and invariants that hold in every game.
"""
import itertools
import math
import os
import subprocess
import sys
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from positions import (COUNTS, LAKES, T, TYPES, board, header, make_record, sq,
                       start_square, unpack_pieces)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FLAG, BOMB, SCOUT = T["Flag"], T["Bomb"], T["Scout"]


def engine_from(recs, seed=1, **kw):
    recs = np.stack(recs) if isinstance(recs, (list, tuple)) else recs
    return O.OracleEngine.from_records(recs, seed, **kw)


# ---------------------------------------------------------------- battle
def test_battle_table_matches_paper_fixture():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "battle_table.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 10
    code = {"A": 0, "D": 1, "T": 2}
    ties = 0
    for a, row in enumerate(rows):
        assert row[0] == TYPES[a]
        for d, sym in enumerate(row[1:]):
            assert O.battle(a, d) == code[sym], (TYPES[a], TYPES[d])
            ties += sym == "T"
    assert ties == 10
    # the Spy/Marshal asymmetry: attacker decides
    assert O.battle(T["Spy"], T["Marshal"]) == 0 and O.battle(T["Marshal"], T["Spy"]) == 0


# ---------------------------------------------------------------- geometry, setup
def test_board_geometry_fresh_setup():
    e = O.OracleEngine(64, seed=7)
    rec = e.export()
    for g in range(64):
        b = board(rec[g])
        assert sum(1 for s in range(100) if b[s] != -2) == 92          # App. A: 92 squares
        lakes = {s for s in range(100) if b[s] == -2}
        assert lakes == LAKES and {99 - s for s in lakes} == lakes
        pcs = unpack_pieces(rec[g])
        for pid in range(80):
            p = pcs[pid]
            assert p["alive"] == 1 and p["revealed"] == 0 and p["moved"] == 0
            s = start_square(pid)
            assert b[s] == pid
            row = s // 10
            assert (row <= 3) if pid < 40 else (row >= 6)
        for owner in (0, 1):
            c = Counter(pcs[pid]["type"] for pid in range(owner * 40, owner * 40 + 40))
            assert [c[t] for t in range(12)] == COUNTS                   # Table pieces


def test_setup_shuffle_uniform():
    # every slot receives each type with probability count/40
    n = 20000
    counts = np.zeros((40, 12))
    for g in range(n):
        t = O.setup_types(3, g, 0, g & 1)
        counts[np.arange(40), t] += 1
    expect = n * np.array(COUNTS) / 40.0
    for slot in (0, 13, 39):
        chi2 = ((counts[slot] - expect) ** 2 / expect).sum()
        assert chi2 < 45.0, (slot, chi2)      # 11 dof; p ~ 4e-6


# ---------------------------------------------------------------- Philox
def _kat_rows():
    rows = []
    for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if l.strip() and not l.startswith("#"):
            v = [int(x, 16) for x in l.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, expect in _kat_rows():
        assert O.philox4x32_10(ctr, key).tolist() == expect


def test_philox_against_independent_library(tmp_path):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    hdr = os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")
    if not os.path.exists(hdr):
        pytest.skip("PyTorch Philox header not installed")
    src = tmp_path / "phx.cpp"
    src.write_text(r'''
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int a = 1; a + 5 < argc; a += 6) {
    uint32_t v[6];
    for (int i = 0; i < 6; i++) v[i] = (uint32_t)strtoul(argv[a + i], 0, 16);
    at::philox_engine e((uint64_t)v[4] | ((uint64_t)v[5] << 32),
                        (uint64_t)v[2] | ((uint64_t)v[3] << 32),
                        (uint64_t)v[0] | ((uint64_t)v[1] << 32));
    for (int i = 0; i < 4; i++) printf("%08x ", e());
    printf("\n");
  }
}
''')
    exe = tmp_path / "phx"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I" + inc, str(src), "-o", str(exe)])
    rng = np.random.default_rng(0)
    cases = rng.integers(0, 2 ** 32, size=(64, 6), dtype=np.uint64)
    args = [format(int(x), "08x") for x in cases.ravel()]
    out = subprocess.check_output([str(exe)] + args).decode().split("\n")
    for i in range(64):
        c = cases[i]
        mine = O.philox4x32_10(c[0:4], c[4:6]).tolist()
        assert mine == [int(x, 16) for x in out[i].split()]


# ---------------------------------------------------------------- legal moves
def brute_legal(b, types, player):
    """All (from, to) pairs checked one by one against App. A's movement rule."""
    out = set()
    for f in range(100):
        pid = b[f]
        if pid < 0 or pid // 40 != player:
            continue
        t = types[pid]
        if t in (FLAG, BOMB):
            continue
        rf, cf = divmod(f, 10)
        for to in range(100):
            if to == f or b[to] == -2:
                continue
            if b[to] >= 0 and b[to] // 40 == player:
                continue
            rt, ct = divmod(to, 10)
            if rf != rt and cf != ct:
                continue
            dist = abs(rf - rt) + abs(cf - ct)
            if t != SCOUT and dist != 1:
                continue
            if rf == rt:
                between = [rf * 10 + c for c in range(min(cf, ct) + 1, max(cf, ct))]
            else:
                between = [r * 10 + cf for r in range(min(rf, rt) + 1, max(rf, rt))]
            if any(b[x] != -1 for x in between):
                continue
            out.add(100 * f + to)
    return out


def random_position(rng, n_red, n_blue):
    squares = [s for s in range(100) if s not in LAKES]
    chosen = rng.choice(squares, size=n_red + n_blue, replace=False)
    pieces = []
    for i, s in enumerate(chosen):
        owner = 0 if i < n_red else 1
        pieces.append(dict(sq=int(s), owner=owner, type=int(rng.integers(0, 12)),
                           revealed=int(rng.integers(0, 2))))
    # keep per-owner type counts within the Table so ids can be assigned
    for owner in (0, 1):
        c = Counter()
        for p in pieces:
            if p["owner"] == owner:
                while c[p["type"]] >= COUNTS[p["type"]]:
                    p["type"] = (p["type"] + 1) % 12
                c[p["type"]] += 1
    return make_record(pieces, ply=int(rng.integers(0, 2)))


def test_legal_moves_brute_force_random_positions():
    rng = np.random.default_rng(11)
    recs = [random_position(rng, int(rng.integers(1, 41)), int(rng.integers(1, 41)))
            for _ in range(150)]
    e = engine_from(recs)
    for g, rec in enumerate(recs):
        b = board(rec)
        types = [p["type"] for p in unpack_pieces(rec)]
        for player in (0, 1):
            n, legal = e.legal_list(g, player)
            got = set(np.flatnonzero(legal).tolist())
            assert got == brute_legal(b, types, player)
            assert n == len(got)


def test_legal_moves_brute_force_played_games():
    e = O.OracleEngine(48, seed=5, max_moves=1000)
    for ply in range(180):
        e.ply(obs=False)
        if ply % 30 == 29:
            rec = e.export()
            for g in range(48):
                b = board(rec[g])
                types = [p["type"] for p in unpack_pieces(rec[g])]
                for player in (0, 1):
                    n, legal = e.legal_list(g, player)
                    assert set(np.flatnonzero(legal).tolist()) == brute_legal(b, types, player)


def test_initial_legal_count_closed_form():
    # only the six front squares next to the lanes can move at ply 0: a Scout has
    # 3 moves (2 empty squares + an attack on row 6), other movable pieces 1.
    e = O.OracleEngine(500, seed=9)
    m, nl = e.mask()
    rec = e.export()
    for g in range(500):
        pcs = unpack_pieces(rec[g])
        b = board(rec[g])
        expect = 0
        for c in (0, 1, 4, 5, 8, 9):
            t = pcs[b[sq(3, c)]]["type"]
            expect += 0 if t in (FLAG, BOMB) else (3 if t == SCOUT else 1)
        assert nl[g] == expect
        assert int(sum(bin(int(w)).count("1") for w in m[g])) == expect


def test_lone_scout_has_18_moves():
    for s in (sq(0, 0), sq(2, 4), sq(7, 9), sq(9, 5), sq(3, 8)):
        rec = make_record([dict(sq=s, owner=0, type="Scout")])
        e = engine_from([rec])
        n, legal = e.legal_list(0, 0)
        assert n == 18


def test_long_moves_mark_a_known_scout():
    # App. A: only a Scout moves more than one square; such a move is public
    rec = make_record([dict(sq=sq(1, 0), owner=0, type="Scout"), dict(sq=sq(1, 9), owner=0, type="Scout"),
                       dict(sq=sq(8, 0), owner=1, type="Scout"), dict(sq=sq(0, 0), owner=0, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Flag")])
    e = engine_from([rec])
    far, near = int(board(rec)[10]), int(board(rec)[19])
    _step(e, 100 * 10 + 40)          # (1,0) -> (4,0): three squares
    _step(e, 100 * 80 + 70)          # blue one square
    _step(e, 100 * 19 + 29)          # (1,9) -> (2,9): one square
    pcs = unpack_pieces(e.export()[0])
    assert pcs[far]["long_move"] == 1 and pcs[far]["moved"] == 1 and pcs[far]["revealed"] == 0
    assert pcs[near]["long_move"] == 0 and pcs[near]["moved"] == 1
    blue = int(board(rec)[80])
    assert pcs[blue]["long_move"] == 0


def _step(e, action):
    r = e.step(np.array([action], dtype=np.int16))
    assert r["first_bad"] == -1, action


def test_scout_blocked_by_lake_piece_and_range_attack():
    # Scout at (4,0): east is blocked after (4,1) by the lake at (4,2)
    rec = make_record([dict(sq=sq(4, 0), owner=0, type="Scout"),
                       dict(sq=sq(8, 0), owner=1, type="Bomb"),
                       dict(sq=sq(1, 0), owner=0, type="Flag")])
    e = engine_from([rec])
    n, legal = e.legal_list(0, 0)
    got = {(a // 100, a % 100) for a in np.flatnonzero(legal)}
    expect = {(40, 41), (40, 50), (40, 60), (40, 70), (40, 80), (40, 30), (40, 20)}
    assert got == expect


# ---------------------------------------------------------------- terminal logic
def step_one(rec, action, **kw):
    e = engine_from([rec], **kw)
    r = e.step(np.array([action], dtype=np.int16))
    return r, e.export()[0]


def test_terminal_flag_capture():
    rec = make_record([dict(sq=sq(3, 0), owner=0, type="Scout"),
                       dict(sq=sq(6, 0), owner=1, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Scout"),
                       dict(sq=sq(0, 9), owner=0, type="Flag")], battleless=99)
    r, out = step_one(rec, 100 * 30 + 60)
    assert r["done"][0] == 1 and r["outcome"][0] == 1 and r["reason"][0] == 1
    assert r["ep_len"][0] == 1
    h = header(out)
    assert h["done"] == 1 and h["battleless"] == 0


def test_terminal_forced_win_and_draw():
    # blue keeps only immovable pieces: after red's move blue cannot move -> red wins
    base = [dict(sq=sq(8, 8), owner=1, type="Bomb"), dict(sq=sq(9, 9), owner=1, type="Flag"),
            dict(sq=sq(0, 0), owner=0, type="Flag")]
    rec = make_record(base + [dict(sq=sq(3, 3), owner=0, type="Major")])
    r, _ = step_one(rec, 100 * 33 + 34)
    assert (r["done"][0], r["outcome"][0], r["reason"][0]) == (1, 1, 2)
    # red's last movable piece dies on a Bomb: neither side can move -> draw
    rec = make_record(base + [dict(sq=sq(7, 8), owner=0, type="Major")])
    r, out = step_one(rec, 100 * 78 + 88)
    assert (r["done"][0], r["outcome"][0], r["reason"][0]) == (1, 0, 3)
    # blue to act with no moves while red can move: red wins even before a move
    rec = make_record(base + [dict(sq=sq(3, 3), owner=0, type="Major")], ply=1)
    e = engine_from([rec])
    e.terminal_check(0)
    h = header(e.export()[0])
    assert (h["done"], h["outcome"], h["reason"]) == (1, 1, 2)


def test_terminal_k_move_and_max_moves_priority():
    pcs = [dict(sq=sq(3, 3), owner=0, type="Major"), dict(sq=sq(6, 6), owner=1, type="Major"),
           dict(sq=sq(0, 0), owner=0, type="Flag"), dict(sq=sq(9, 9), owner=1, type="Flag")]
    r, _ = step_one(make_record(pcs, battleless=99, ply=10), 100 * 33 + 34)
    assert (r["done"][0], r["outcome"][0], r["reason"][0]) == (1, 0, 4)
    r, _ = step_one(make_record(pcs, battleless=5, ply=998), 100 * 33 + 34, max_moves=999)
    assert (r["done"][0], r["outcome"][0], r["reason"][0]) == (1, 0, 5)
    # k-move before max-moves on the same ply
    r, _ = step_one(make_record(pcs, battleless=99, ply=998), 100 * 33 + 34, max_moves=999)
    assert r["reason"][0] == 4
    r, _ = step_one(make_record(pcs, battleless=98, ply=10), 100 * 33 + 34)
    assert r["done"][0] == 0


def test_illegal_action_leaves_game_unchanged():
    rec = make_record([dict(sq=sq(3, 3), owner=0, type="Major"),
                       dict(sq=sq(6, 6), owner=1, type="Major")])
    e = engine_from([rec])
    before = e.export()
    r = e.step(np.array([100 * 33 + 53], dtype=np.int16))
    assert r["first_bad"] == 0
    assert np.array_equal(before, e.export())


# ---------------------------------------------------------------- battles, deaths
@pytest.mark.parametrize("att,dfd,rdef,res,catt,cdef", [
    ("Sergeant", "Bomb", 0, "D", 3, 0),
    ("Lieutenant", "Lieutenant", 1, "T", 2, 5),
    ("Lieutenant", "Lieutenant", 0, "T", 3, 6),
    ("Captain", "Major", 1, "D", 1, 0),
    ("Major", "Captain", 1, "A", 0, 4),
    ("Major", "Captain", 0, "A", 0, 6),
    ("Spy", "Marshal", 0, "A", 0, 6),
    ("Marshal", "Spy", 1, "A", 0, 4),
    ("Miner", "Bomb", 1, "A", 0, 4),
])
def test_battle_deaths_and_reveal(att, dfd, rdef, res, catt, cdef):
    rec = make_record([dict(sq=sq(4, 4), owner=0, type=att),
                       dict(sq=sq(5, 4), owner=1, type=dfd, revealed=rdef),
                       dict(sq=sq(0, 0), owner=0, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Flag"),
                       dict(sq=sq(9, 0), owner=1, type="Scout"),
                       dict(sq=sq(0, 9), owner=0, type="Scout")], battleless=7)
    ida, idd = board(rec)[44], board(rec)[54]
    r, out = step_one(rec, 100 * 44 + 54)
    pcs = unpack_pieces(out)
    b = board(out)
    A, D = pcs[ida], pcs[idd]
    assert A["revealed"] == 1 and D["revealed"] == 1 and A["moved"] == 1
    assert header(out)["battleless"] == 0
    assert b[44] == -1
    assert b[54] == {"A": ida, "D": idd, "T": -1}[res]
    assert A["alive"] == (res == "A") and D["alive"] == (res == "D")
    assert A["death_cause"] == catt and D["death_cause"] == cdef
    if not A["alive"]:
        assert A["death_square"] == 54
    if not D["alive"]:
        assert D["death_square"] == 54


# ---------------------------------------------------------------- history scenarios
# Expected bits below follow the written readings of App. C.1 (threat = the
# mover ends next to an enemy piece; evasion = a threatened piece steps to an
# empty square away from the threatener; active adjacency = an attack that was
# available and not taken; protection = a non-battle reply in which the mover
# newly becomes adjacent to a square next to the threatener).  The paper has no
# worked example: these pins depend on those readings.
HID = 10


def run_and_pieces(rec, action):
    r, out = step_one(rec, action)
    return unpack_pieces(out), board(rec), out


def nonzero_history(p):
    return {k: p[k] for k in ("threat", "evade", "adj", "prot", "prot_against", "been_by",
                              "been_against") if p[k]}


def test_threat_hidden_and_revealed_and_bomb_skipped():
    rec = make_record([dict(sq=sq(0, 0), owner=0, type="Scout"),
                       dict(sq=sq(5, 0), owner=1, type="Colonel", revealed=1),
                       dict(sq=sq(4, 1), owner=1, type="Bomb", revealed=1),
                       dict(sq=sq(9, 9), owner=1, type="Flag"),
                       dict(sq=sq(0, 9), owner=0, type="Flag")])
    scout = board(rec)[0]
    pcs, _, _ = run_and_pieces(rec, 100 * 0 + 40)
    assert nonzero_history(pcs[scout]) == {"threat": 1 << T["Colonel"]}
    rec = make_record([dict(sq=sq(0, 0), owner=0, type="Scout"),
                       dict(sq=sq(4, 1), owner=1, type="Bomb"),
                       dict(sq=sq(9, 9), owner=1, type="Flag"),
                       dict(sq=sq(0, 9), owner=0, type="Flag")])
    pcs, _, _ = run_and_pieces(rec, 40)
    assert nonzero_history(pcs[board(rec)[0]]) == {"threat": 1 << HID}


def test_evasion_adjacency_and_empty_square_protection():
    # blue's hidden Major moved 51 -> 41 on the previous ply, next to red's Captain
    rec = make_record([dict(sq=sq(3, 1), owner=0, type="Captain"),
                       dict(sq=sq(4, 1), owner=1, type="Major", moved=1),
                       dict(sq=sq(0, 9), owner=0, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Flag")],
                      ply=2, moves=[(5, 15), (51, 41)])
    cap, maj = board(rec)[31], board(rec)[41]
    pcs, _, _ = run_and_pieces(rec, 100 * 31 + 30)
    # evaded the hidden Major, skipped attacking it, and now guards empty (4,0)
    assert nonzero_history(pcs[cap]) == {"evade": 1 << HID, "adj": 1 << HID,
                                         "prot": 1 << 11, "prot_against": 1 << 12}
    assert nonzero_history(pcs[maj]) == {}


def test_attacking_the_threatener_is_not_an_evasion():
    # blue's hidden Major moved next to red's Captain; the Captain attacks it
    rec = make_record([dict(sq=sq(3, 1), owner=0, type="Captain"),
                       dict(sq=sq(4, 1), owner=1, type="Major", moved=1),
                       dict(sq=sq(0, 9), owner=0, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Flag")],
                      ply=2, moves=[(5, 15), (51, 41)])
    cap = board(rec)[31]
    pcs, _, _ = run_and_pieces(rec, 100 * 31 + 41)
    assert pcs[cap]["alive"] == 0 and pcs[cap]["death_cause"] == 3
    assert pcs[cap]["evade"] == 0 and pcs[cap]["adj"] == 0


def test_protection_of_a_piece_against_revealed_general():
    rec = make_record([dict(sq=sq(3, 4), owner=0, type="Sergeant"),
                       dict(sq=sq(2, 5), owner=0, type="Captain"),
                       dict(sq=sq(4, 4), owner=1, type="General", revealed=1, moved=1),
                       dict(sq=sq(0, 9), owner=0, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Flag")],
                      ply=2, moves=[(3, 13), (54, 44)])
    sgt, cap = board(rec)[34], board(rec)[25]
    pcs, _, _ = run_and_pieces(rec, 100 * 25 + 35)
    G = T["General"]
    assert nonzero_history(pcs[cap]) == {"prot": (1 << 12) | (1 << 11), "prot_against": 1 << G}
    assert nonzero_history(pcs[sgt]) == {"adj": 1 << G, "been_by": 1 << 12,
                                         "been_against": 1 << G}


def test_no_protection_after_a_non_threat():
    # the previous blue move ended next to no red piece: not a threat
    rec = make_record([dict(sq=sq(2, 5), owner=0, type="Captain"),
                       dict(sq=sq(4, 4), owner=1, type="General", revealed=1, moved=1),
                       dict(sq=sq(0, 9), owner=0, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Flag")],
                      ply=2, moves=[(3, 13), (54, 44)])
    pcs, _, _ = run_and_pieces(rec, 100 * 25 + 35)
    assert nonzero_history(pcs[board(rec)[25]]) == {}


def test_winning_attacker_threatens_and_adjacency_excludes_chosen_attack():
    rec = make_record([dict(sq=sq(4, 4), owner=0, type="Marshal"),
                       dict(sq=sq(5, 4), owner=1, type="Captain"),
                       dict(sq=sq(6, 4), owner=1, type="Spy", revealed=1),
                       dict(sq=sq(4, 5), owner=1, type="Scout", revealed=1),
                       dict(sq=sq(0, 9), owner=0, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Flag")])
    mar = board(rec)[44]
    pcs, _, _ = run_and_pieces(rec, 100 * 44 + 54)
    # pre-move: the Scout at (4,5) could have been attacked -> adjacency (revealed Scout);
    # post-move on (5,4): next to the revealed Spy at (6,4) -> threat
    assert nonzero_history(pcs[mar]) == {"adj": 1 << T["Scout"], "threat": 1 << T["Spy"]}


# ---------------------------------------------------------------- encoding
PROB_PLY0 = [6, 51, 32, 26, 26, 26, 19, 13, 6, 6, 6, 38]   # round(255 * count / 40)


def test_probability_channels_at_ply0():
    e = O.OracleEngine(8, seed=2)
    obs = e.encode()
    for g in range(8):
        for o in (0, 1):
            x = obs[g, o].reshape(488, 100)
            enemy = [f for f in range(100) if f >= 60]          # enemy rows in own frame
            own = [f for f in range(100) if f < 40]
            for t in range(12):
                assert (x[12 + t, enemy] == PROB_PLY0[t]).all()
                assert (x[24 + t, own] == PROB_PLY0[t]).all()
                assert (x[12 + t, own] == 0).all() and (x[24 + t, enemy] == 0).all()
            assert PROB_PLY0 == [math.floor(255 * c / 40 + 0.5) for c in COUNTS]


def enumerate_marginals(types, moved, long_move=None):
    """Exact marginals by enumerating every distinct assignment of the unknown
    types to the unrevealed pieces that gives no moved piece a Flag or Bomb and
    every piece seen moving more than one square the Scout type (App. A: only
    Scouts move further than one square)."""
    long_move = long_move or [0] * len(types)
    tally = [Counter() for _ in types]
    total = 0
    for perm in set(itertools.permutations(types)):
        if any(m and t in (FLAG, BOMB) for t, m in zip(perm, moved)):
            continue
        if any(lm and t != SCOUT for t, lm in zip(perm, long_move)):
            continue
        total += 1
        for i, t in enumerate(perm):
            tally[i][t] += 1
    return [{t: Fraction(c[t], total) for t in range(12)} for c in tally]


def test_probability_channels_brute_force_enumeration():
    rng = np.random.default_rng(4)
    for trial in range(60):
        h = int(rng.integers(2, 8))
        pool = [t for t in range(12) for _ in range(COUNTS[t])]
        types = [int(x) for x in rng.choice(pool, size=h, replace=False)]
        moved = [int(t not in (FLAG, BOMB) and rng.integers(0, 2)) for t in types]
        # some moved Scouts were seen moving more than one square
        long_move = [int(m and t == SCOUT and rng.integers(0, 2)) for t, m in zip(types, moved)]
        squares = rng.choice([s for s in range(60, 100)], size=h, replace=False)
        pieces = [dict(sq=int(s), owner=1, type=t, moved=m, long_move=lm)
                  for s, t, m, lm in zip(squares, types, moved, long_move)]
        pieces += [dict(sq=sq(0, 0), owner=0, type="Flag"),
                   dict(sq=sq(0, 1), owner=0, type="Scout", revealed=1)]
        # a few revealed blue pieces that must not disturb the hidden multiset
        if trial % 3 == 0:
            pieces.append(dict(sq=sq(4, 5), owner=1, type="Miner", revealed=1))
        rec = make_record(pieces)
        e = engine_from([rec])
        marg = enumerate_marginals(types, moved, long_move)
        x = e.encode()[0, 0].reshape(488, 100)       # red observes blue
        y = e.encode()[0, 1].reshape(488, 100)       # blue observes its own pieces via 24-35
        for i, s in enumerate(squares):
            for t in range(12):
                if long_move[i]:
                    p = Fraction(int(t == SCOUT))     # a known Scout
                else:
                    num, den = O.hidden_prob(e, 0, 1, moved[i], t)
                    p = Fraction(num, den) if den else Fraction(0)
                assert p == marg[i][t]
                q = math.floor(255 * p + Fraction(1, 2))
                assert x[12 + t, int(s)] == q
                assert y[24 + t, 99 - int(s)] == q
        if trial % 3 == 0:
            assert x[12 + T["Miner"], 45] == 255


def test_encoding_invariants_during_play():
    e = O.OracleEngine(32, seed=13, max_moves=1000, auto_reset=True)
    pads = [275, 288, 301, 327, 340, 353, 455]
    for ply in range(260):
        if ply % 37 == 36:
            obs = e.encode()
            rec = e.export()
            for g in range(32):
                b = board(rec[g])
                pcs = unpack_pieces(rec[g])
                hd = header(rec[g])
                for o in (0, 1):
                    x = obs[g, o].reshape(488, 100).astype(int)
                    fr = (lambda s: s) if o == 0 else (lambda s: 99 - s)
                    own_alive = sum(1 for p in pcs[o * 40:o * 40 + 40] if p["alive"])
                    assert x[0:12].sum() == own_alive
                    dead = [p for p in pcs if not p["alive"] and p["type"] != FLAG]
                    assert x[109:131].sum() == len(dead)
                    assert (x[pads] == 0).all()
                    occ = [fr(s) for s in range(100) if b[s] >= 0]
                    assert (x[355:455].sum(axis=0)[occ] == 1).all()
                    assert x[355:455].sum() == len(occ)
                    assert x[38].sum() == sum(1 for s in range(100) if b[s] == -1)
                    for i in range(32):
                        plane = x[456 + i]
                        if i < hd["ring_count"]:
                            assert (plane == 1).sum() == 1 and (plane == 255).sum() == 1
                        else:
                            assert plane.sum() == 0
                    # probability rows: each hidden square's exact probabilities sum to 1
                    for s in range(100):
                        pid = b[s]
                        if pid < 0 or pcs[pid]["revealed"] or pcs[pid]["long_move"]:
                            continue
                        w = pid // 40
                        tot = Fraction(0)
                        for t in range(12):
                            num, den = O.hidden_prob(e, g, w, pcs[pid]["moved"], t)
                            tot += Fraction(num, den) if den else 0
                        assert tot == 1
                # conservation: board <-> alive pieces, lakes never entered
                alive_ids = sorted(p["id"] for p in pcs if p["alive"])
                assert sorted(int(v) for v in b if v >= 0) == alive_ids
                assert all(b[s] == -2 for s in LAKES)
                assert all(p["revealed"] for p in pcs if not p["alive"])
                for p in pcs:
                    if p["type"] in (FLAG, BOMB):
                        assert p["threat"] == p["evade"] == p["adj"] == 0
                        assert p["prot"] == p["prot_against"] == p["been_by"] == 0 or \
                            p["type"] == BOMB and p["prot"] == p["prot_against"] == 0
        e.ply(obs=False)


def test_record_round_trip_and_determinism():
    a = O.OracleEngine(40, seed=21, auto_reset=True)
    b = O.OracleEngine(40, seed=21, auto_reset=True)
    for _ in range(150):
        ra, rb = a.ply(obs=False), b.ply(obs=False)
        assert np.array_equal(ra["actions"], rb["actions"])
    rec = a.export()
    c = O.OracleEngine.from_records(rec, 21, auto_reset=True)
    assert np.array_equal(c.export(), rec)
    assert np.array_equal(c.encode(), a.encode())


def test_sampling_picks_rth_legal_action_uniformly():
    e = O.OracleEngine(200, seed=31)
    hits = []
    for _ in range(30):
        m, nl = e.mask()
        a = e.sample(m, nl)
        rec = e.export()
        for g in range(200):
            legal = [x for x in range(10000) if int(m[g][x >> 6]) >> (x & 63) & 1]
            if not legal:
                assert a[g] == -1 and header(rec[g])["done"] == 1
                continue
            assert a[g] in legal
            hits.append((len(legal), legal.index(int(a[g]))))
        e.step(a)
    # given n legal actions, the chosen rank is uniform on 0..n-1: pooled chi-square
    chi2, dof = 0.0, 0
    for n in set(h[0] for h in hits):
        ranks = [r for (m, r) in hits if m == n]
        if len(ranks) < 5 * n:
            continue
        c = np.bincount(ranks, minlength=n)
        exp = len(ranks) / n
        chi2 += ((c - exp) ** 2 / exp).sum()
        dof += n - 1
    assert dof > 20
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


# ---------------------------------------------------------------- resampling
def test_resample_invariants_and_observer_obs_unchanged():
    e = O.OracleEngine(64, seed=17, max_moves=1000)
    for _ in range(100):
        e.ply(obs=False)
    rec = e.export()
    alive = [g for g in range(64) if header(rec[g])["done"] == 0][:8]
    src = O.OracleEngine.from_records(rec[alive], 17, max_moves=1000)
    per = 16
    rs = src.resample(per, seed=17)
    out = rs.export()
    obs_src = src.encode()
    obs_rs = rs.encode()
    for i in range(len(alive)):
        ps = unpack_pieces(rec[alive[i]])
        for j in range(per):
            k = i * per + j
            assert header(out[k])["game_id"] == k
            pr = unpack_pieces(out[k])
            assert Counter(p["type"] for p in pr[40:]) == Counter(p["type"] for p in ps[40:])
            for pid in range(80):
                if pid < 40 or ps[pid]["revealed"] or not ps[pid]["alive"] or ps[pid]["long_move"]:
                    assert pr[pid]["type"] == ps[pid]["type"]
                if pr[pid]["moved"] and pr[pid]["alive"]:
                    assert pr[pid]["type"] not in (FLAG, BOMB)
            assert np.array_equal(obs_rs[k, 0], obs_src[i, 0])


def test_resample_frequencies_match_probability_channels():
    e = O.OracleEngine(8, seed=23, max_moves=1000)
    for _ in range(100):
        e.ply(obs=False)
    rec = e.export()
    g = [i for i in range(8) if header(rec[i])["done"] == 0][0]
    src = O.OracleEngine.from_records(rec[[g]], 23, max_moves=1000)
    per = 6000
    rs = src.resample(per, seed=99)
    out = rs.export()
    ps = unpack_pieces(rec[g])
    hidden = [pid for pid in range(40, 80) if ps[pid]["alive"] and not ps[pid]["revealed"]]
    types = np.array([[int(out[k][256 + 16 * pid]) & 15 for pid in hidden] for k in range(per)])
    for col, pid in enumerate(hidden[:12]):
        for t in range(12):
            if ps[pid]["long_move"]:
                p = float(t == SCOUT)                 # a known Scout keeps its type
            else:
                num, den = O.hidden_prob(src, 0, 1, ps[pid]["moved"], t)
                p = num / den if den else 0.0
            f = (types[:, col] == t).mean()
            assert abs(f - p) < 5 * math.sqrt(max(p * (1 - p), 1e-9) / per) + 1e-9, (pid, t, f, p)


# ---------------------------------------------------------------- two-square rule
# App. A: a piece may not cross the same square boundary on more than three
# consecutive turns of its owner.  The oracle tracks each player's last-moved
# piece and the squares it occupied (App. B.2).
def _play(e, actions):
    for a in actions:
        r = e.step(np.array([a], dtype=np.int16))
        assert r["first_bad"] == -1, a
    return r


def _moves_of(e, frm):
    n, legal = e.legal_list(0, e.export()[0][8] & 1)
    return {int(a) % 100 for a in np.flatnonzero(legal) if int(a) // 100 == frm}


def _corridor_position():
    # red Sergeant on (3,0); blue Scout on (9,9) moving elsewhere
    return make_record([dict(sq=sq(3, 0), owner=0, type="Sergeant"),
                        dict(sq=sq(0, 9), owner=0, type="Flag"),
                        dict(sq=sq(9, 9), owner=1, type="Scout"),
                        dict(sq=sq(9, 0), owner=1, type="Flag")])


def test_two_square_fourth_crossing_is_forbidden():
    A, B = sq(3, 0), sq(4, 0)
    b1, b2 = sq(9, 9), sq(9, 8)
    seq = [100 * A + B, 100 * b1 + b2, 100 * B + A, 100 * b2 + b1, 100 * A + B, 100 * b1 + b2]
    on = engine_from([_corridor_position()], two_square=True)
    _play(on, seq[:4])
    assert B in _moves_of(on, A)             # the third crossing is still allowed
    _play(on, seq[4:])
    assert _moves_of(on, B) == {sq(5, 0), sq(4, 1)}   # back to A would be the fourth
    off = engine_from([_corridor_position()], two_square=False)
    _play(off, seq)
    assert _moves_of(off, B) == {A, sq(5, 0), sq(4, 1)}
    # the record keeps the state; an import continues with it
    rec = on.export()[0]
    assert list(rec[24:30]) == [rec[64 + B], 4, A, B, A, B]
    again = engine_from([rec], two_square=True)
    assert _moves_of(again, B) == {sq(5, 0), sq(4, 1)}
    # the rule is reported, and only with the flag on
    assert on.two_square_applies(0) and not off.two_square_applies(0)


def test_two_square_resets_when_another_piece_moves():
    A, B = sq(3, 0), sq(4, 0)
    rec = make_record([dict(sq=A, owner=0, type="Sergeant"), dict(sq=sq(0, 5), owner=0, type="Miner"),
                       dict(sq=sq(0, 9), owner=0, type="Flag"), dict(sq=sq(9, 9), owner=1, type="Scout"),
                       dict(sq=sq(9, 0), owner=1, type="Flag")])
    e = engine_from([rec], two_square=True)
    blue = [100 * (99 - k) + 98 - k for k in range(4)]   # the blue Scout walks west along row 9
    _play(e, [100 * A + B, blue[0], 100 * B + A, blue[1], 100 * sq(0, 5) + sq(0, 4), blue[2],
              100 * A + B, blue[3]])
    assert A in _moves_of(e, B)
    assert not e.two_square_applies(0)


def test_two_square_scout_spans():
    # a Scout on column 0 (no lakes): 30 -> 60 -> 40 -> 70 crosses row
    # boundaries {3,4,5}, {4,5}, {4,5,6}; boundaries 4 and 5 were crossed on
    # all three turns, so from 70 any move crossing 4 or 5 is forbidden
    rec = make_record([dict(sq=sq(3, 0), owner=0, type="Scout"), dict(sq=sq(0, 9), owner=0, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Scout"), dict(sq=sq(9, 5), owner=1, type="Flag")])
    e = engine_from([rec], two_square=True)
    b1, b2 = sq(9, 9), sq(9, 8)
    _play(e, [100 * 30 + 60, 100 * b1 + b2, 100 * 60 + 40, 100 * b2 + b1, 100 * 40 + 70, 100 * b1 + b2])
    got = _moves_of(e, 70)
    row7 = {sq(7, c) for c in range(1, 10)}
    assert got == {60, 80, 90} | row7
    e_off = engine_from([rec], two_square=False)
    _play(e_off, [100 * 30 + 60, 100 * b1 + b2, 100 * 60 + 40, 100 * b2 + b1, 100 * 40 + 70, 100 * b1 + b2])
    assert _moves_of(e_off, 70) == {0, 10, 20, 30, 40, 50, 60, 80, 90} | row7
    # a turn along another line breaks the run: 30 -> 60 -> 40 -> 41 restricts nothing
    e2 = engine_from([rec], two_square=True)
    _play(e2, [100 * 30 + 60, 100 * b1 + b2, 100 * 60 + 40, 100 * b2 + b1, 100 * 40 + 41, 100 * b1 + b2])
    n_on, _ = e2.legal_list(0, 0, two_square=True)
    n_off, _ = e2.legal_list(0, 0, two_square=False)
    assert n_on == n_off


def test_two_square_can_leave_no_legal_move():
    # the red Sergeant shuttles in a dead end walled by its own Bombs: after
    # three crossings it has no move left and red loses (forced win for blue)
    walls = [dict(sq=s, owner=0, type="Bomb") for s in (sq(0, 1), sq(1, 1), sq(2, 0))]
    pieces = [dict(sq=sq(0, 0), owner=0, type="Sergeant"), dict(sq=sq(0, 9), owner=0, type="Flag")] + walls + [
        dict(sq=sq(9, 9), owner=1, type="Scout"), dict(sq=sq(9, 0), owner=1, type="Flag")]
    rec = make_record(pieces)
    A, B = sq(0, 0), sq(1, 0)
    b1, b2 = sq(9, 9), sq(9, 8)
    seq = [100 * A + B, 100 * b1 + b2, 100 * B + A, 100 * b2 + b1, 100 * A + B, 100 * b1 + b2]
    on = engine_from([rec], two_square=True)
    r = _play(on, seq)
    assert r["done"][0] == 1 and r["outcome"][0] == -1 and r["reason"][0] == 2
    off = engine_from([rec], two_square=False)
    r = _play(off, seq)
    assert r["done"][0] == 0


# ---------------------------------------------------------------- magnet policy and search policy
# Section 2.4 / App. D.4: the magnet policy rho picks a movable piece uniformly
# at random, then one of its legal moves uniformly at random.  App. D.7: the
# search plays pi_search = argmax <q, pi> - alpha KL(pi, rho) - beta KL(pi, pi_theta).
def _replicate(rec, n):
    recs = np.repeat(rec[None], n, axis=0).copy()
    recs[:, 0:4] = np.arange(n, dtype=np.uint32).view(np.uint8).reshape(n, 4)   # game ids 0..n-1
    return recs


def _two_piece_position():
    # red Sergeant boxed in to 2 moves, red Scout with a long column, blue far away
    return make_record([dict(sq=sq(0, 0), owner=0, type="Sergeant"), dict(sq=sq(0, 1), owner=0, type="Bomb"),
                        dict(sq=sq(2, 5), owner=0, type="Scout"), dict(sq=sq(0, 9), owner=0, type="Flag"),
                        dict(sq=sq(9, 9), owner=1, type="Flag"), dict(sq=sq(9, 0), owner=1, type="Bomb")])


def test_magnet_probabilities_closed_form():
    e = engine_from([make_record([dict(sq=sq(2, 4), owner=0, type="Scout")]), _two_piece_position()])
    acts, nl = e.legal_actions_list()
    rho = e.magnet()
    assert nl[0] == 18 and np.all(rho[0, :18] == np.float32(1.0 / 18)) and np.all(rho[0, 18:] == 0)
    k = int(nl[1])
    frm = acts[1, :k] // 100
    sergeant = frm == sq(0, 0)
    assert sergeant.sum() == 1                     # only (1,0): (0,1) holds its own Bomb
    scout_moves = int((frm == sq(2, 5)).sum())
    assert np.all(rho[1, :k][sergeant] == np.float32(1 / 2))
    assert np.all(rho[1, :k][~sergeant] == np.float32(1.0) / np.float32(2 * scout_moves))
    assert abs(float(rho[1].sum()) - 1.0) < 1e-6
    assert np.all(acts[1, k:] == -1) and list(acts[1, :k]) == sorted(acts[1, :k])


def test_magnet_sampler_is_uniform_over_pieces_then_moves():
    from scipy.stats import chisquare
    n = 6000
    rec = _two_piece_position()
    e = O.OracleEngine.from_records(_replicate(rec, n), seed=13, sampler=O.SAMPLER_MAGNET)
    m, nl = e.mask()
    a = e.sample(m, nl)
    frm = a // 100
    assert set(np.unique(frm)) == {sq(0, 0), sq(2, 5)}
    n_sgt = int((frm == sq(0, 0)).sum())
    assert chisquare([n_sgt, n - n_sgt]).pvalue > 1e-3          # pieces equally likely
    scout = a[frm == sq(2, 5)]
    _, counts = np.unique(scout, return_counts=True)
    assert chisquare(counts).pvalue > 1e-3                     # moves of the Scout equally likely
    u = O.OracleEngine.from_records(_replicate(rec, n), seed=13)   # the uniform sampler for contrast
    ua = u.sample(*u.mask())
    assert (ua // 100 == sq(0, 0)).mean() < 0.2


def _objective(pi, q, rho, pth, alpha, beta):
    kl = lambda p, r: float(np.sum(np.where(p > 0, p * np.log(np.where(p > 0, p, 1) / r), 0.0)))
    return float(np.dot(q, pi)) - alpha * kl(pi, rho) - beta * kl(pi, pth)


def test_search_policy_maximises_the_regularised_objective():
    rng = np.random.default_rng(5)
    recs = [_two_piece_position(), make_record([dict(sq=sq(2, 4), owner=0, type="Scout"),
                                                dict(sq=sq(7, 7), owner=1, type="Flag")])]
    e = engine_from(recs)
    acts, nl = e.legal_actions_list()
    rho = e.magnet().astype(np.float64)
    for alpha, beta in ((0.002, 0.02), (0.5, 0.3), (1.0, 0.0)):
        q = np.zeros((2, 256), np.float32)
        lp = np.zeros((2, 256), np.float32)
        pth = []
        for g in range(2):
            k = int(nl[g])
            q[g, :k] = rng.uniform(-1, 1, k)
            logits = rng.normal(0, 1, k)
            lp[g, :k] = logits - np.log(np.exp(logits).sum())
            pth.append(np.exp(lp[g, :k].astype(np.float64)))
        pi = e.mmd(q, lp, alpha, beta)
        for g in range(2):
            k = int(nl[g])
            p = pi[g, :k]
            assert abs(p.sum() - 1) < 1e-12 and np.all(pi[g, k:] == 0)
            best = _objective(p, q[g, :k].astype(np.float64), rho[g, :k], pth[g], alpha, beta)
            for _ in range(300):   # no other point of the simplex does better
                r = rng.dirichlet(np.ones(k) * rng.uniform(0.2, 5))
                mix = rng.uniform(0, 1)
                cand = mix * r + (1 - mix) * p
                assert _objective(cand, q[g, :k].astype(np.float64), rho[g, :k], pth[g], alpha, beta) <= best + 1e-12


def test_search_policy_special_cases():
    e = engine_from([_two_piece_position()])
    acts, nl = e.legal_actions_list()
    k = int(nl[0])
    rho = e.magnet()
    q = np.zeros((1, 256), np.float32)
    lp = np.zeros((1, 256), np.float32)
    lp[0, :k] = np.log(rho[0, :k].astype(np.float64))
    # q = 0 and pi_theta = rho: the regularisers agree, so pi = rho
    assert np.allclose(e.mmd(q, lp, 0.002, 0.02)[0, :k], rho[0, :k], rtol=1e-6)
    # a large advantage on one action with weak regularisation takes almost all mass
    q[0, 3] = 1.0
    assert e.mmd(q, lp, 0.002, 0.02)[0, 3] > 0.999


def test_policy_sampler_follows_the_given_distribution():
    from scipy.stats import chisquare
    n = 8000
    rec = _two_piece_position()
    e = O.OracleEngine.from_records(_replicate(rec, n), seed=3)
    acts, nl = e.legal_actions_list()
    k = int(nl[0])
    probs = np.zeros((n, 256), np.float32)
    w = np.arange(1, k + 1, dtype=np.float64)
    w[2] = 0.0                                   # a zero-weight action is never played
    probs[:, :k] = (w / w.sum()).astype(np.float32)
    a = e.sample_policy(probs)
    idx = np.searchsorted(acts[0, :k], a)
    assert np.all(acts[0, idx] == a) and not np.any(idx == 2)
    counts = np.bincount(idx, minlength=k).astype(np.float64)
    keep = w > 0
    assert chisquare(counts[keep], f_exp=n * w[keep] / w.sum()).pvalue > 1e-3
    one = np.zeros((n, 256), np.float32)
    one[:, 5] = 1.0
    assert np.all(e.sample_policy(one) == acts[0, 5])


# ---------------------------------------------------------------- continuous-chasing rule
# App. A: a chasing player may not make a threat that recreates a position of
# the chase, unless the moved piece returns to the square it held before that
# player's previous turn.  Table "chase": threat, evade, chase.
_CHASE = [1112, 1303, 1202, 313, 203, 1312, 302, 1213]   # red Captain chases the blue Lieutenant


def _chase_position():
    return make_record([dict(sq=11, owner=0, type="Captain"), dict(sq=25, owner=0, type="Major"),
                        dict(sq=13, owner=1, type="Lieutenant"),
                        dict(sq=sq(0, 9), owner=0, type="Flag"), dict(sq=sq(9, 0), owner=1, type="Flag")])


def test_chasing_rule_forbids_a_repeated_position():
    on = engine_from([_chase_position()], chasing=True)
    off = engine_from([_chase_position()], chasing=False)
    lens = []
    for a in _CHASE:
        _play(on, [a])
        _play(off, [a])
        lens.append(int(on.export()[0][40]))
    assert lens == [1, 2, 3, 4, 5, 6, 7, 8] and on.export()[0][41] == 0
    # 02 -> 12 threatens the Lieutenant on 13 and recreates the position after
    # the chase's first threat (Captain 12, Major 25, Lieutenant 13)
    assert 12 not in _moves_of(on, 2) and 12 in _moves_of(off, 2)
    # 02 -> 03 recreates the position after the third threat, but returns the
    # Captain to the square it held before red's previous turn: allowed
    assert 3 in _moves_of(on, 2)
    assert on.chase_applies(0) and not off.chase_applies(0)
    # the chase state travels with the record
    again = engine_from([on.export()[0]], chasing=True)
    assert 12 not in _moves_of(again, 2)


def test_chasing_rule_compares_positions_with_the_same_side_to_move():
    # A red Scout circles 20 -> 22 -> 21 while a blue Lieutenant steps 32 -> 31
    # -> 32 away from it; a blue Bomb on 30 keeps 20 a threat square.  Each red
    # move is a threat and each blue move an evasion, so after four plies the
    # chase has length 4 and red is to move.  The threat 21 -> 20 recreates the
    # board of the chase's start, but there red was to move and after the
    # threat blue is: not the same position, so the move stays legal.
    def position():
        return make_record([dict(sq=20, owner=0, type="Scout"), dict(sq=32, owner=1, type="Lieutenant"),
                            dict(sq=30, owner=1, type="Bomb"), dict(sq=sq(7, 9), owner=0, type="Flag"),
                            dict(sq=sq(9, 0), owner=1, type="Flag")])
    on = engine_from([position()], chasing=True, k_battleless=1000)
    _play(on, [2022, 3231, 2221, 3132])
    assert int(on.export()[0][40]) == 4 and int(on.export()[0][41]) == 0
    assert 20 in _moves_of(on, 21)
    b0 = [int(v) for v in board(position())]
    res = [int(v) for v in board(on.export()[0])]
    res[20], res[21] = res[21], -1
    assert res == b0                      # the board would indeed repeat


def _loop(cols):
    """The border of rows 0-3 x cols 0..cols-1, in walking order."""
    return ([sq(0, c) for c in range(cols)] + [sq(r, cols - 1) for r in (1, 2, 3)] +
            [sq(3, c) for c in range(cols - 2, -1, -1)] + [sq(r, 0) for r in (2, 1)])


@pytest.mark.parametrize("cols,forbidden", [(6, True), (7, False)])
def test_chasing_rule_window_is_the_32_ply_move_record(cols, forbidden):
    # A red Captain follows a blue Lieutenant around a loop of squares, one step
    # behind it: every red move threatens, every blue move evades, so the chase
    # grows by one each ply.  Around a 16-square loop (cols 0-5) the position
    # after red's first threat comes back 31 plies later, inside the 32 plies
    # the move record keeps: forbidden.  Around an 18-square loop (cols 0-6) it
    # comes back after 35 plies, beyond the record: the rule does not see it.
    loop = _loop(cols)
    n = len(loop)
    rec = make_record([dict(sq=loop[0], owner=0, type="Captain"), dict(sq=loop[2], owner=1, type="Lieutenant"),
                       dict(sq=sq(7, 9), owner=0, type="Flag"), dict(sq=sq(9, 0), owner=1, type="Flag")])
    e = engine_from([rec], chasing=True, k_battleless=1000)
    for i in range(n):
        _play(e, [100 * loop[i] + loop[(i + 1) % n], 100 * loop[(i + 2) % n] + loop[(i + 3) % n]])
    assert int(e.export()[0][40]) == 2 * n and int(e.export()[0][41]) == 0
    assert (loop[1] not in _moves_of(e, loop[0])) == forbidden


def test_chase_ends_on_a_battle_or_a_non_evasion():
    e = engine_from([_chase_position()], chasing=True)
    _play(e, _CHASE[:3])
    assert e.export()[0][40] == 3
    # the Lieutenant on 03 attacks the Captain on 02 instead of evading: the battle ends the chase
    r = e.step(np.array([100 * 3 + 2], np.int16))
    assert r["first_bad"] == -1 and e.export()[0][40] == 0
    e2 = engine_from([_chase_position()], chasing=True)
    _play(e2, _CHASE[:1])
    # 13 -> 14 leaves the Captain's side but stays... 14 is not next to 12, so it
    # is an evasion; 13 -> 23 likewise; the Flag cannot move, so blue breaks the
    # chase only with a move of another piece: give blue a Scout for that
    assert e2.export()[0][40] == 1


def _is_threat(b, p, x, y):
    """Non-battle move x -> y of player p ending next to an enemy piece."""
    if b[y] != -1:
        return False
    res = list(b)
    res[y], res[x] = res[x], -1
    return any(res[z] >= 0 and (res[z] >= 40) != (p == 1) for z in _nbrs(y))


def _nbrs(s):
    r, c = divmod(s, 10)
    return [10 * (r + dr) + c + dc for dr, dc in ((-1, 0), (1, 0), (0, -1), (0, 1))
            if 0 <= r + dr < 10 and 0 <= c + dc < 10]


def chasing_actions(e, rng):
    """A move chooser that keeps chases going: a threat when one exists (else
    an evasion of the last threat, else any legal move), at random among them."""
    recs = e.export()
    out = np.full(e.n, -1, dtype=np.int16)
    for g in range(e.n):
        r = recs[g]
        if r[17]:
            continue
        p = int(r[8]) & 1
        b = [int(v) for v in board(r)]
        _, legal = e.legal_list(g, p)
        acts = [int(a) for a in np.flatnonzero(legal)]
        if not acts:
            continue
        threats = [a for a in acts if _is_threat(b, p, a // 100, a % 100)]
        last = (int(r[8]) - 1) & 31
        a_sq = int(r[164 + 2 * last + 1]) if r[16] else -1
        evades = [a for a in acts if a_sq >= 0 and b[a_sq] >= 0 and a_sq in _nbrs(a // 100)
                  and a_sq not in _nbrs(a % 100) and b[a % 100] == -1]
        pool = threats or evades or acts
        out[g] = pool[int(rng.integers(0, len(pool)))]
    return out


def test_chasing_rule_against_full_board_history():
    """Sparse games driven to chase: the chase state and the forbidden moves
    equal those obtained from the full board history by the definitions of
    Table "chase" (positions of the chase within the last 32 plies, compared
    as whole boards)."""
    rng = np.random.default_rng(17)
    recs = [random_position(rng, int(rng.integers(1, 4)), int(rng.integers(1, 4))) for _ in range(150)]
    e = engine_from(recs, chasing=True, max_moves=400)
    hist = [[[int(v) for v in board(r)]] for r in e.export()]
    state = [(0, 0, None) for _ in recs]     # chase length, chaser, last move (player, from, to)
    seen_forbidden = 0
    for ply in range(120):
        a = chasing_actions(e, rng)
        before = e.export()
        r = e.step(a)
        assert r["first_bad"] == -1
        after = e.export()
        for g in range(len(recs)):
            if a[g] < 0 or before[g][17]:
                continue
            p = int(before[g][8]) & 1
            f, t = divmod(int(a[g]), 100)
            b0 = hist[g][-1]
            b1 = [int(v) for v in board(after[g])]
            battle = b0[t] >= 0
            L, C, last = state[g]
            threat = not battle and any(b1[z] >= 0 and (b1[z] >= 40) != (p == 1) for z in _nbrs(t))
            evade = (not battle and last is not None and last[0] != p and b0[last[2]] >= 0
                     and last[2] in _nbrs(f) and last[2] not in _nbrs(t))
            if not battle and L > 0 and p == C and threat and L % 2 == 0:
                L += 1
            elif not battle and L > 0 and p != C and evade and L % 2 == 1:
                L += 1
            elif threat:
                L, C = 1, p
            else:
                L, C = 0, 0
            L = min(L, 255)
            state[g] = (L, C, (p, f, t))
            hist[g].append(b1)
            assert (int(after[g][40]), int(after[g][41])) == (L, C), (g, ply)
            if after[g][17]:
                continue
            q = 1 - p
            _, l_on = e.legal_list(g, q)
            _, l_off = e.legal_list(g, q, chasing=False)
            got = set(np.flatnonzero(l_off & ~l_on).tolist())
            want = set()
            if L >= 2 and L % 2 == 0 and C == q:
                # positions of the chase within the 32-ply record with the same
                # side to move as the one a threat creates: an odd number of plies back
                window = [hist[g][-1 - k] for k in range(1, min(L, 32) + 1) if k % 2 == 1]
                prev = (int(after[g][8]) - 2) & 31
                prev_f, prev_t = int(after[g][164 + 2 * prev]), int(after[g][165 + 2 * prev])
                for act in np.flatnonzero(l_off):
                    x, y = divmod(int(act), 100)
                    if not _is_threat(b1, q, x, y) or (prev_t == x and prev_f == y):
                        continue
                    res = list(b1)
                    res[y], res[x] = res[x], -1
                    if any(res == w for w in window):
                        want.add(int(act))
            assert got == want, (g, ply, got, want)
            seen_forbidden += len(want)
    print("forbidden moves seen:", seen_forbidden)
    assert seen_forbidden >= 20, seen_forbidden


def test_acting_player_encoding_is_the_acting_observer_of_both():
    # App. B.1: ComputeInfostateTensor returns the acting player's information state
    both = O.OracleEngine(40, seed=12, auto_reset=True)
    act = O.OracleEngine(40, seed=12, auto_reset=True, acting_obs=True)
    for ply in range(25):
        pre = both.export()[:, 8] & 1      # acting player of the pre-move state the obs show
        rb, ra = both.ply(obs=True), act.ply(obs=True)
        assert ra["obs"].shape == (40, 1, 488, 10, 10)
        assert np.array_equal(ra["obs"][:, 0], rb["obs"][np.arange(40), pre])
