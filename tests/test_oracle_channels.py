"""Channel placement of the oracle's information-state encoder (no GPU).

Each test builds a position by hand, encodes it with the oracle and compares
whole channel groups against planes written out by hand from the paper's
channel tables (App. C.1 "Representation of the Board State", App. C.2
"Representation of recent moves").  The expected entries below are literal
(observer, channel, row, column, value) tuples in the observer's frame; the
comment beside each says which table row it follows.  Nothing here calls the
encoder to produce an expectation.

Frames (reading R4): red (observer 0) sees absolute squares; blue (observer 1)
sees the board rotated by 180 degrees, so absolute (r, c) appears at
(9 - r, 9 - c).  Every failure message names the observer and the channel.
"""
import numpy as np

import oracle as O
from positions import DEFAULT_TYPE, LAKES, T, make_record, sq, start_square

RED, BLUE = 0, 1


def engine_from(recs, seed=1, **kw):
    return O.OracleEngine.from_records(np.stack(recs), seed, **kw)


def encode(rec, **kw):
    """Both observers' planes of one record, as int [2][488][100]."""
    return engine_from([rec], **kw).encode()[0].reshape(2, 488, 100).astype(int)


def planes(entries):
    """Zero planes with the listed (observer, channel, row, col, value) set."""
    x = np.zeros((2, 488, 100), dtype=int)
    for o, c, r, col, v in entries:
        assert x[o, c, 10 * r + col] == 0, ("entry listed twice", o, c, r, col)
        x[o, c, 10 * r + col] = v
    return x


def check_group(got, want, channels, what):
    for o in (RED, BLUE):
        for c in channels:
            g, w = got[o, c], want[o, c]
            if not np.array_equal(g, w):
                gs = {divmod(int(f), 10): int(g[f]) for f in np.flatnonzero(g)}
                ws = {divmod(int(f), 10): int(w[f]) for f in np.flatnonzero(w)}
                raise AssertionError(f"{what}: observer {o} channel {c}: got {gs}, expected {ws}")


# ---------------------------------------------------------------- channels 0-11, 36-40
# Red: one piece of each type, Spy..Marshal on row 1 (column = type index),
# Flag on (2,0), Bomb on (2,1).  Blue: Spy..Marshal on row 8 (column = type
# index), Flag on (7,8), Bomb on (7,9).  Revealed: red Miner (1,2), red Marshal
# (1,9), blue Spy (8,0), blue Colonel (8,7).  Moved: red Scout (1,1), red
# General (1,8), red Marshal (1,9), blue Colonel (8,7), blue Captain (8,5).
def _basic_position():
    pcs = []
    for t in range(10):
        pcs.append(dict(sq=sq(1, t), owner=RED, type=t, revealed=int(t in (2, 9)),
                        moved=int(t in (1, 8, 9))))
        pcs.append(dict(sq=sq(8, t), owner=BLUE, type=t, revealed=int(t in (0, 7)),
                        moved=int(t in (5, 7))))
    pcs += [dict(sq=sq(2, 0), owner=RED, type="Flag"), dict(sq=sq(2, 1), owner=RED, type="Bomb"),
            dict(sq=sq(7, 8), owner=BLUE, type="Flag"), dict(sq=sq(7, 9), owner=BLUE, type="Bomb")]
    return make_record(pcs)


def test_channels_own_type_0_to_11():
    got = encode(_basic_position())
    want = []
    # 0-11: the square holds a piece of the observer of type T (channel = type index)
    for t in range(10):
        want.append((RED, t, 1, t, 1))            # red's own row-1 pieces
        want.append((BLUE, t, 1, 9 - t, 1))       # blue's row-8 pieces, rotated to row 1
    want += [(RED, 10, 2, 0, 1), (RED, 11, 2, 1, 1),      # red Flag (2,0), Bomb (2,1)
             (BLUE, 10, 2, 1, 1), (BLUE, 11, 2, 0, 1)]    # blue Flag (7,8) -> (2,1), Bomb (7,9) -> (2,0)
    check_group(got, planes(want), range(0, 12), "own type")


def test_channels_hidden_empty_moved_36_to_40():
    got = encode(_basic_position())
    red_hidden = [(1, c) for c in (0, 1, 3, 4, 5, 6, 7, 8)] + [(2, 0), (2, 1)]
    blue_hidden = [(8, c) for c in (1, 2, 3, 4, 5, 6, 8, 9)] + [(7, 8), (7, 9)]
    rot = lambda rc: (9 - rc[0], 9 - rc[1])
    want = []
    # 36: hidden pieces of the observer; 37: hidden pieces of the opponent
    want += [(RED, 36, r, c, 1) for r, c in red_hidden]
    want += [(RED, 37, r, c, 1) for r, c in blue_hidden]
    want += [(BLUE, 36, *rot(rc), 1) for rc in blue_hidden]
    want += [(BLUE, 37, *rot(rc), 1) for rc in red_hidden]
    # 39: the observer's pieces that moved; 40: the opponent's pieces that moved
    want += [(RED, 39, 1, 1, 1), (RED, 39, 1, 8, 1), (RED, 39, 1, 9, 1)]
    want += [(RED, 40, 8, 5, 1), (RED, 40, 8, 7, 1)]
    want += [(BLUE, 39, 1, 4, 1), (BLUE, 39, 1, 2, 1)]                     # (8,5), (8,7) rotated
    want += [(BLUE, 40, 8, 8, 1), (BLUE, 40, 8, 1, 1), (BLUE, 40, 8, 0, 1)]  # (1,1), (1,8), (1,9)
    # 38: empty squares: neither a lake nor one of the 24 occupied squares (the
    # occupied set is symmetric under the rotation, so both views agree)
    occupied = {sq(1, c) for c in range(10)} | {sq(8, c) for c in range(10)} | \
               {sq(2, 0), sq(2, 1), sq(7, 8), sq(7, 9)}
    for o in (RED, BLUE):
        want += [(o, 38, s // 10, s % 10, 1) for s in range(100) if s not in occupied and s not in LAKES]
    check_group(got, planes(want), range(36, 41), "hidden/empty/moved")


# ---------------------------------------------------------------- channels 41-42
def test_channels_move_fractions_41_42():
    # 41: fraction of the maximum game length used; 42: fraction of the k-move
    # budget used; each as round-half-up(255 x) on all 100 squares (lakes too)
    cases = [(dict(ply=250, battleless=37), dict(max_moves=1000, k_battleless=100), 64, 94),
             (dict(ply=500, battleless=2), dict(max_moves=1000, k_battleless=100), 128, 5),
             (dict(ply=2, battleless=1), dict(max_moves=4000, k_battleless=200), 0, 1)]
    pcs = [dict(sq=sq(0, 0), owner=RED, type="Flag"), dict(sq=sq(9, 9), owner=BLUE, type="Flag")]
    for hdr, cfg, v41, v42 in cases:
        got = encode(make_record(pcs, **hdr), **cfg)
        want = [(o, 41, s // 10, s % 10, v41) for o in (RED, BLUE) for s in range(100)]
        want += [(o, 42, s // 10, s % 10, v42) for o in (RED, BLUE) for s in range(100)]
        check_group(got, planes(want), (41, 42), f"fractions {hdr} {cfg}")


# ---------------------------------------------------------------- channels 43-108
def test_channels_threat_evasion_adjacency_43_to_108():
    # red Captain on (3,4): threatened a revealed Marshal and a hidden piece,
    # evaded a revealed Spy, was actively adjacent to a revealed Scout and a
    # hidden piece.  Blue Lieutenant on (6,2): threatened a revealed General,
    # evaded a hidden piece, was actively adjacent to a revealed Colonel.
    # Slots: type index for Spy..Marshal, 10 for a hidden piece.
    rec = make_record([
        dict(sq=sq(3, 4), owner=RED, type="Captain", threat=(1 << 9) | (1 << 10), evade=1 << 0,
             adj=(1 << 1) | (1 << 10)),
        dict(sq=sq(6, 2), owner=BLUE, type="Lieutenant", threat=1 << 8, evade=1 << 10, adj=1 << 7),
        dict(sq=sq(0, 0), owner=RED, type="Flag"), dict(sq=sq(9, 9), owner=BLUE, type="Flag")])
    got = encode(rec)
    want = [
        # red's view: own piece (43-53 threat, 54-64 evasion, 65-75 adjacency)
        (RED, 52, 3, 4, 1), (RED, 53, 3, 4, 1),        # threatened Marshal (43+9), hidden (53)
        (RED, 54, 3, 4, 1),                            # evaded Spy (54+0)
        (RED, 66, 3, 4, 1), (RED, 75, 3, 4, 1),        # adjacent to Scout (65+1), hidden (75)
        # red's view of the opponent's piece (76-86, 87-97, 98-108)
        (RED, 84, 6, 2, 1),                            # threatened General (76+8)
        (RED, 97, 6, 2, 1),                            # evaded a hidden piece (97)
        (RED, 105, 6, 2, 1),                           # adjacent to Colonel (98+7)
        # blue's view: own Lieutenant at (6,2) -> (3,7)
        (BLUE, 51, 3, 7, 1), (BLUE, 64, 3, 7, 1), (BLUE, 72, 3, 7, 1),
        # blue's view of red's Captain at (3,4) -> (6,5)
        (BLUE, 85, 6, 5, 1), (BLUE, 86, 6, 5, 1), (BLUE, 87, 6, 5, 1),
        (BLUE, 99, 6, 5, 1), (BLUE, 108, 6, 5, 1)]
    check_group(got, planes(want), range(43, 109), "threat/evasion/adjacency")


# ---------------------------------------------------------------- channels 109-250
def _full_board(dead):
    """Every id alive on its start square with its default type, except the dead."""
    gone = {d["id"] for d in dead}
    pcs = [dict(sq=start_square(pid), owner=pid // 40, type=DEFAULT_TYPE[pid % 40], id=pid)
           for pid in range(80) if pid not in gone]
    return make_record(pcs, dead=dead)


# Captured pieces (default types by id: 1 Scout, 9 Miner, 14 Sergeant, 29
# Colonel; blue 40 Spy, 66 Major, 74 Bomb), with cause and death square.
_DEAD = [dict(id=9, cause=1, sq=sq(4, 5)),     # red Miner, start (0,9)
         dict(id=29, cause=4, sq=sq(5, 5)),    # red Colonel, start (2,9)
         dict(id=1, cause=2, sq=sq(4, 0)),     # red Scout, start (0,1)
         dict(id=14, cause=5, sq=sq(4, 1)),    # red Sergeant, start (1,4)
         dict(id=40, cause=6, sq=sq(3, 3)),    # blue Spy, start 99 = (9,9)
         dict(id=66, cause=3, sq=sq(5, 9)),    # blue Major, start 99-26 = (7,3)
         dict(id=74, cause=6, sq=sq(6, 5))]    # blue Bomb, start 99-34 = (6,5)


def test_channels_captured_start_squares_109_to_130():
    got = encode(_full_board(_DEAD))
    # 109-119: the observer's captured pieces of type Spy..Marshal, Bomb at their
    # start square (slot = type index, 10 for the Bomb); 120-130: the opponent's
    want = [(RED, 111, 0, 9, 1), (RED, 116, 2, 9, 1), (RED, 110, 0, 1, 1), (RED, 112, 1, 4, 1),
            (RED, 120, 9, 9, 1), (RED, 126, 7, 3, 1), (RED, 130, 6, 5, 1),
            (BLUE, 109, 0, 0, 1), (BLUE, 115, 2, 6, 1), (BLUE, 119, 3, 4, 1),
            (BLUE, 122, 9, 0, 1), (BLUE, 127, 7, 0, 1), (BLUE, 121, 9, 8, 1), (BLUE, 123, 8, 5, 1)]
    check_group(got, planes(want), range(109, 131), "captured pieces")


def test_channels_causes_of_death_131_to_250():
    got = encode(_full_board(_DEAD))
    # 131 + 10 (cause - 1) + type: where the observer's Spy..Marshal died and why;
    # 191 + ... the same for the opponent.  A dead Bomb has no death channel.
    want = [(RED, 133, 4, 5, 1),     # Miner, cause 1: 131 + 0 + 2
            (RED, 168, 5, 5, 1),     # Colonel, cause 4: 131 + 30 + 7
            (RED, 142, 4, 0, 1),     # Scout, cause 2: 131 + 10 + 1
            (RED, 174, 4, 1, 1),     # Sergeant, cause 5: 131 + 40 + 3
            (RED, 241, 3, 3, 1),     # blue Spy, cause 6: 191 + 50 + 0
            (RED, 217, 5, 9, 1),     # blue Major, cause 3: 191 + 20 + 6
            (BLUE, 181, 6, 6, 1),    # own Spy at (3,3) -> (6,6)
            (BLUE, 157, 4, 0, 1),    # own Major at (5,9) -> (4,0)
            (BLUE, 193, 5, 4, 1),    # red Miner at (4,5) -> (5,4)
            (BLUE, 228, 4, 4, 1),    # red Colonel at (5,5) -> (4,4)
            (BLUE, 202, 5, 9, 1),    # red Scout at (4,0) -> (5,9)
            (BLUE, 234, 5, 8, 1)]    # red Sergeant at (4,1) -> (5,8)
    check_group(got, planes(want), range(131, 251), "causes of death")


# ---------------------------------------------------------------- channels 251-354
def test_channels_protection_251_to_354():
    # Slots of the four 13-channel groups: type index for Spy..Marshal, 10 for a
    # Bomb, 11 for an empty square (protected only; a padding plane otherwise),
    # 12 for a hidden piece.
    rec = make_record([
        dict(sq=sq(3, 4), owner=RED, type="Major",
             prot=(1 << 0) | (1 << 10) | (1 << 11) | (1 << 12), prot_against=(1 << 9) | (1 << 12),
             been_by=1 << 1, been_against=(1 << 8) | (1 << 12)),
        dict(sq=sq(6, 6), owner=BLUE, type="Captain", prot=1 << 3, prot_against=1 << 10,
             been_by=1 << 12, been_against=1 << 0),
        dict(sq=sq(0, 0), owner=RED, type="Flag"), dict(sq=sq(9, 9), owner=BLUE, type="Flag")])
    got = encode(rec)
    want = [
        # red's own Major: protected Spy (251), Bomb (261), an empty square (262),
        # a hidden piece (263); against a Marshal (264+9) and a hidden piece (276);
        # was protected by a Scout (277+1); against a General (290+8), hidden (302)
        (RED, 251, 3, 4, 1), (RED, 261, 3, 4, 1), (RED, 262, 3, 4, 1), (RED, 263, 3, 4, 1),
        (RED, 273, 3, 4, 1), (RED, 276, 3, 4, 1), (RED, 278, 3, 4, 1),
        (RED, 298, 3, 4, 1), (RED, 302, 3, 4, 1),
        # the opponent's Captain (+52): protected a Sergeant (303+3), against a
        # Bomb (316+10), protected by a hidden piece (329+12), against a Spy (342)
        (RED, 306, 6, 6, 1), (RED, 326, 6, 6, 1), (RED, 341, 6, 6, 1), (RED, 342, 6, 6, 1),
        # blue's view: own Captain at (6,6) -> (3,3)
        (BLUE, 254, 3, 3, 1), (BLUE, 274, 3, 3, 1), (BLUE, 289, 3, 3, 1), (BLUE, 290, 3, 3, 1),
        # blue's view of the red Major at (3,4) -> (6,5)
        (BLUE, 303, 6, 5, 1), (BLUE, 313, 6, 5, 1), (BLUE, 314, 6, 5, 1), (BLUE, 315, 6, 5, 1),
        (BLUE, 325, 6, 5, 1), (BLUE, 328, 6, 5, 1), (BLUE, 330, 6, 5, 1),
        (BLUE, 350, 6, 5, 1), (BLUE, 354, 6, 5, 1)]
    check_group(got, planes(want), range(251, 355), "protection")


# ---------------------------------------------------------------- channels 355-455
def test_channels_start_square_355_to_455():
    # channel 355 + k marks the square of the piece that started on square k
    # (k in the observer's frame); 455 stays zero.  Ids: red 5 (start 5) now on
    # (3,5); red 39 (start 39) on its start square; blue 52 (start 87) on (5,0);
    # blue 45 (start 94) on (6,1).
    rec = make_record([dict(sq=sq(3, 5), owner=RED, type="Scout", id=5),
                       dict(sq=sq(3, 9), owner=RED, type="Bomb", id=39),
                       dict(sq=sq(5, 0), owner=BLUE, type="Miner", id=52),
                       dict(sq=sq(6, 1), owner=BLUE, type="Scout", id=45)])
    got = encode(rec)
    want = [(RED, 360, 3, 5, 1), (RED, 394, 3, 9, 1), (RED, 442, 5, 0, 1), (RED, 449, 6, 1, 1),
            # blue: start k -> 99 - k, square s -> 99 - s
            (BLUE, 449, 6, 4, 1),    # start 5 -> 94; (3,5) -> (6,4)
            (BLUE, 415, 6, 0, 1),    # start 39 -> 60; (3,9) -> (6,0)
            (BLUE, 367, 4, 9, 1),    # start 87 -> 12; (5,0) -> (4,9)
            (BLUE, 360, 3, 8, 1)]    # start 94 -> 5; (6,1) -> (3,8)
    check_group(got, planes(want), range(355, 456), "start squares")


# ---------------------------------------------------------------- channels 456-487
def test_channels_recent_moves_most_recent_first():
    # App. C.2: one plane per recent move, +1 (0x01) at the destination and -1
    # (0xFF) at the source; plane 456 is the most recent move.
    pcs = [dict(sq=sq(3, 1), owner=RED, type="Scout"), dict(sq=sq(7, 8), owner=BLUE, type="Scout"),
           dict(sq=sq(0, 0), owner=RED, type="Flag"), dict(sq=sq(9, 9), owner=BLUE, type="Flag")]
    moves = [(1, 11), (98, 88), (11, 21), (88, 78), (21, 31)]   # oldest first
    got = encode(make_record(pcs, ply=5, moves=moves))
    F = 0xFF
    want = [(RED, 456, 3, 1, 1), (RED, 456, 2, 1, F), (BLUE, 456, 6, 8, 1), (BLUE, 456, 7, 8, F),   # 21->31
            (RED, 457, 7, 8, 1), (RED, 457, 8, 8, F), (BLUE, 457, 2, 1, 1), (BLUE, 457, 1, 1, F),   # 88->78
            (RED, 458, 2, 1, 1), (RED, 458, 1, 1, F), (BLUE, 458, 7, 8, 1), (BLUE, 458, 8, 8, F),   # 11->21
            (RED, 459, 8, 8, 1), (RED, 459, 9, 8, F), (BLUE, 459, 1, 1, 1), (BLUE, 459, 0, 1, F),   # 98->88
            (RED, 460, 1, 1, 1), (RED, 460, 0, 1, F), (BLUE, 460, 8, 8, 1), (BLUE, 460, 9, 8, F)]   # 1->11
    check_group(got, planes(want), range(456, 488), "recent moves")


def test_channels_recent_moves_across_the_ring_wrap():
    # 32 moves made at plies 8..39 (move k: square k -> k + 10); the ring slot of
    # ply t is t mod 32, so the most recent (ply 39, 31 -> 41) sits in slot 7.
    pcs = [dict(sq=sq(0, 0), owner=RED, type="Flag"), dict(sq=sq(9, 9), owner=BLUE, type="Flag")]
    moves = [(k, k + 10) for k in range(32)]
    got = encode(make_record(pcs, ply=40, moves=moves))
    want = []
    for i in range(32):
        f, t = 31 - i, 41 - i            # plane 456 + i: the move of ply 39 - i
        want += [(RED, 456 + i, t // 10, t % 10, 1), (RED, 456 + i, f // 10, f % 10, 0xFF),
                 (BLUE, 456 + i, (99 - t) // 10, (99 - t) % 10, 1),
                 (BLUE, 456 + i, (99 - f) // 10, (99 - f) % 10, 0xFF)]
    check_group(got, planes(want), range(456, 488), "recent moves (wrapped ring)")


# ---------------------------------------------------------------- channels 12-35
def test_channels_probabilities_of_known_and_single_hidden_pieces():
    # Red: revealed Spy on (1,1); hidden unmoved Flag on (0,0); every other red
    # piece captured (hence revealed), so red's unknown multiset is {Flag}: P = 1.
    # Blue: hidden moved Marshal on (8,8), revealed Bomb on (9,9); the rest
    # captured: blue's unknown multiset is {Marshal}: P = 1.
    rec = make_record([dict(sq=sq(1, 1), owner=RED, type="Spy", revealed=1),
                       dict(sq=sq(0, 0), owner=RED, type="Flag"),
                       dict(sq=sq(8, 8), owner=BLUE, type="Marshal", moved=1),
                       dict(sq=sq(9, 9), owner=BLUE, type="Bomb", revealed=1)])
    got = encode(rec)
    # 12-23: the opponent's piece on the square has type T; 24-35: the same for
    # the observer's own pieces, from the opponent's point of view; 255 = certain
    want = [(RED, 12 + 9, 8, 8, 255), (RED, 12 + 11, 9, 9, 255),
            (RED, 24 + 0, 1, 1, 255), (RED, 24 + 10, 0, 0, 255),
            (BLUE, 12 + 0, 8, 8, 255), (BLUE, 12 + 10, 9, 9, 255),
            (BLUE, 24 + 9, 1, 1, 255), (BLUE, 24 + 11, 0, 0, 255)]
    check_group(got, planes(want), range(12, 36), "probabilities")


def test_channels_probabilities_of_moved_and_unmoved_hidden_pieces():
    # Blue's unknown pieces: an unmoved Flag (9,0), an unmoved Miner (9,1) and a
    # moved Captain (7,5).  The four assignments with no Flag on the moved piece
    # are equally likely: (F, Ca | Mi), (Ca, F | Mi), (F, Mi | Ca), (Mi, F | Ca).
    # Unmoved squares: Flag 1/2 -> 128, Miner 1/4 -> 64, Captain 1/4 -> 64.
    # Moved square: Miner 1/2 -> 128, Captain 1/2 -> 128.
    rec = make_record([dict(sq=sq(9, 0), owner=BLUE, type="Flag"),
                       dict(sq=sq(9, 1), owner=BLUE, type="Miner"),
                       dict(sq=sq(7, 5), owner=BLUE, type="Captain", moved=1),
                       dict(sq=sq(0, 0), owner=RED, type="Flag", revealed=1)])
    got = encode(rec)
    FL, MI, CA = 12 + T["Flag"], 12 + T["Miner"], 12 + T["Captain"]
    want = [(RED, FL, 9, 0, 128), (RED, MI, 9, 0, 64), (RED, CA, 9, 0, 64),
            (RED, FL, 9, 1, 128), (RED, MI, 9, 1, 64), (RED, CA, 9, 1, 64),
            (RED, MI, 7, 5, 128), (RED, CA, 7, 5, 128),
            (RED, 24 + T["Flag"], 0, 0, 255),
            # blue's own pieces seen by red: channels 24-35 of blue's view, rotated
            (BLUE, FL + 12, 0, 9, 128), (BLUE, MI + 12, 0, 9, 64), (BLUE, CA + 12, 0, 9, 64),
            (BLUE, FL + 12, 0, 8, 128), (BLUE, MI + 12, 0, 8, 64), (BLUE, CA + 12, 0, 8, 64),
            (BLUE, MI + 12, 2, 4, 128), (BLUE, CA + 12, 2, 4, 128),
            (BLUE, 12 + T["Flag"], 9, 9, 255)]
    check_group(got, planes(want), range(12, 36), "probabilities")


def test_channels_probabilities_with_a_known_scout():
    # As above, plus a blue piece on (7,7) that was seen moving more than one
    # square in one move: only a Scout can (App. A), so it is a known Scout
    # (255 on the Scout channel), and it leaves the unknown set, so the other
    # three squares keep the values of the previous position.
    rec = make_record([dict(sq=sq(9, 0), owner=BLUE, type="Flag"),
                       dict(sq=sq(9, 1), owner=BLUE, type="Miner"),
                       dict(sq=sq(7, 5), owner=BLUE, type="Captain", moved=1),
                       dict(sq=sq(7, 7), owner=BLUE, type="Scout", moved=1, long_move=1),
                       dict(sq=sq(0, 0), owner=RED, type="Flag", revealed=1)])
    got = encode(rec)
    FL, MI, CA, SC = 12 + T["Flag"], 12 + T["Miner"], 12 + T["Captain"], 12 + T["Scout"]
    want = [(RED, FL, 9, 0, 128), (RED, MI, 9, 0, 64), (RED, CA, 9, 0, 64),
            (RED, FL, 9, 1, 128), (RED, MI, 9, 1, 64), (RED, CA, 9, 1, 64),
            (RED, MI, 7, 5, 128), (RED, CA, 7, 5, 128), (RED, SC, 7, 7, 255),
            (RED, 24 + T["Flag"], 0, 0, 255),
            (BLUE, FL + 12, 0, 9, 128), (BLUE, MI + 12, 0, 9, 64), (BLUE, CA + 12, 0, 9, 64),
            (BLUE, FL + 12, 0, 8, 128), (BLUE, MI + 12, 0, 8, 64), (BLUE, CA + 12, 0, 8, 64),
            (BLUE, MI + 12, 2, 4, 128), (BLUE, CA + 12, 2, 4, 128), (BLUE, SC + 12, 2, 2, 255),
            (BLUE, 12 + T["Flag"], 9, 9, 255)]
    check_group(got, planes(want), range(12, 36), "probabilities with a known Scout")
    # the known Scout is still unrevealed: it stays on the hidden channels 36/37
    check_group(got, planes([(RED, 37, r, c, 1) for r, c in ((9, 0), (9, 1), (7, 5), (7, 7))] +
                            [(BLUE, 36, 9 - r, 9 - c, 1) for r, c in ((9, 0), (9, 1), (7, 5), (7, 7))]),
                (36, 37), "hidden pieces")
