"""The oracle's two-square rule against a brute force over the move record.

App. A forbids a piece to cross the same square boundary on more than three
consecutive turns of its owner (App. B.2 keeps the last four squares of each
player's last-acting piece).  The oracle keeps an incremental per-player
record of that piece and its squares (reading R30).  This test rebuilds the
same run from nothing but the move record of the position (the last moves
of the player to move, two plies apart, the opponent's in between ignored)
and the board, and derives which moves the rule removes:

* the run is the player's last three moves if each started where the
  previous one ended and the piece still stands where the last one ended
  (a piece that died in an attack ends its run);
* a move along a row or column crosses the unit boundaries between
  consecutive squares of its segment (a Scout's long move crosses several);
* a move of that piece is removed when it and the three moves of the run all
  cross one boundary.

Over random games with the rule on, the oracle's legal moves must be exactly
the basic rules' legal moves minus those.
"""
import numpy as np

import oracle as O
from positions import board, header


def boundaries(a, b):
    ra, ca = divmod(a, 10)
    rb, cb = divmod(b, 10)
    if ra == rb:
        lo, hi = sorted((ca, cb))
        return {("row", ra, k) for k in range(lo, hi)}
    assert ca == cb, (a, b)
    lo, hi = sorted((ra, rb))
    return {("col", ca, k) for k in range(lo, hi)}


def recorded_move(rec, ply):
    slot = ply & 31
    return int(rec[164 + 2 * slot]), int(rec[164 + 2 * slot + 1])


def removed_moves(rec, legal):
    """Moves of the basic rules' legal set that the two-square rule removes."""
    h = header(rec)
    t, p = h["ply"], h["ply"] & 1
    if h["ring_count"] < 6:
        return set()
    m1, m2, m3 = (recorded_move(rec, t - 2 * k) for k in (1, 2, 3))
    piece = board(rec)[m1[1]]
    if piece < 0 or (piece >= 40) != (p == 1):
        return set()                                   # the run's piece died
    if m2[1] != m1[0] or m3[1] != m2[0]:
        return set()                                   # not one piece's three moves in a row
    common = boundaries(*m3) & boundaries(*m2) & boundaries(*m1)
    return {a for a in legal if a // 100 == m1[1] and boundaries(m1[1], a % 100) & common}


def test_two_square_rule_matches_brute_force_over_random_games():
    n, plies = 48, 300
    eng = O.OracleEngine(n, 23, k_battleless=100, max_moves=1000, auto_reset=False, two_square=True)
    restricted = checked = 0
    for _ in range(plies):
        recs = eng.export()
        for g in range(n):
            h = header(recs[g])
            if h["done"]:
                continue
            p = h["ply"] & 1
            _, base = eng.legal_list(g, p, two_square=False)
            _, ruled = eng.legal_list(g, p, two_square=True)
            base_set = set(np.flatnonzero(base).tolist())
            gone = removed_moves(recs[g], base_set)
            assert set(np.flatnonzero(ruled).tolist()) == base_set - gone, (
                f"game {g} ply {h['ply']}: the oracle removes "
                f"{sorted(base_set - set(np.flatnonzero(ruled).tolist()))}, the brute force {sorted(gone)}")
            restricted += bool(gone)
            checked += 1
        eng.ply(obs=False, mask=False)
    assert checked > 8000
    assert restricted > 0, "no position in the sample had a move removed"
