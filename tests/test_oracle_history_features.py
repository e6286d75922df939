"""The oracle's history features against a brute force over whole games.

App. C.1 defines the per-piece history channels (threat, evasion, active
adjacency, protection) in words, and the paper gives no worked example of
them.  The oracle keeps them as bits in each piece's record words, updated
incrementally inside its step.  This test recomputes, for every ply of many
random games, which bits that ply must add, from nothing but the boards
before and after the move, the pieces' types and reveal flags, and the move
record, following the readings written down for these channels:

* R15 active adjacency: before the move, every movable piece of the mover's
  side next to an enemy piece (which it could attack) notes that enemy,
  except for the pair of the move actually made;
* R14 evasion: when the previous mover A still stands on its destination a,
  a mover next to a that moves to an empty square not next to a notes A;
* R13 threat: a mover that stands on its destination after the move notes
  every enemy piece next to it;
* R16 protection: a non-battle reply to a threat by A (some piece of the
  mover's side was next to a) makes the mover note every square next to a
  that it newly becomes adjacent to (an own piece B there also notes the
  mover and A; an empty square is noted as such);
* R17 reveal flags: before the move for adjacency and evasion, after it for
  threats and protection;

with the slot conventions of the records: Spy..Marshal by type when
revealed, 10 for a hidden piece, revealed Bombs and Flags no slot (threat,
evasion, adjacency); Spy..Marshal by type, Bomb 10, empty 11, hidden 12
(protection).  Every ply of every game must change every piece's history
bits by exactly those increments, and leave them alone otherwise.  The
brute force shares no code with the oracle: it reads the records with the
test package's field decoder and walks squares in plain Python.
"""

import numpy as np

import oracle as O
from positions import LAKES, board, header, make_record, sq, unpack_pieces

FLAG, BOMB = 10, 11
FIELDS = ("threat", "evade", "adj", "prot", "prot_against", "been_by", "been_against")


def neighbours(s):
    r, c = divmod(s, 10)
    out = []
    if r > 0:
        out.append(s - 10)
    if r < 9:
        out.append(s + 10)
    if c > 0:
        out.append(s - 1)
    if c < 9:
        out.append(s + 1)
    return out


def owner(pid):
    return 0 if pid < 40 else 1


def slot_seen(p):
    """Threat, evasion and adjacency slot of a piece, or None."""
    if not p["revealed"]:
        return 10
    return p["type"] if p["type"] < FLAG else None


def slot_guard(p):
    """Protection slot of a piece."""
    if not p["revealed"]:
        return 12
    if p["type"] == BOMB:
        return 10
    assert p["type"] < FLAG, "a revealed Flag ends the game"
    return p["type"]


def expected_increments(pre, post, action):
    """Bits the ply must add, per piece id: {id: {field: bits}}."""
    inc = {}

    def add(pid, field, bit):
        inc.setdefault(pid, {}).setdefault(field, 0)
        inc[pid][field] |= 1 << bit

    h = header(pre)
    b0, b1 = board(pre), board(post)
    p0, p1 = unpack_pieces(pre), unpack_pieces(post)
    me = h["ply"] & 1
    frm, to = divmod(int(action), 100)
    x = b0[frm]
    assert x >= 0 and owner(x) == me
    battle = b0[to] >= 0

    # R15: pre-move adjacency of the mover's movable pieces
    for s in range(100):
        pid = b0[s]
        if pid < 0 or owner(pid) != me or p0[pid]["type"] >= FLAG:
            continue
        for y in neighbours(s):
            e = b0[y]
            if e < 0 or owner(e) == me or (s == frm and y == to):
                continue
            sl = slot_seen(p0[e])
            if sl is not None:
                add(pid, "adj", sl)

    # the previous move's mover, if it still stands on its destination
    A, a = None, None
    if h["ring_count"] > 0:
        last = (h["ply"] - 1) & 31
        a = int(pre[164 + 2 * last + 1])
        if b0[a] >= 0 and owner(b0[a]) != me:
            A = b0[a]

    # R14: evasion
    if A is not None and frm in neighbours(a) and not battle and to not in neighbours(a):
        sl = slot_seen(p0[A])
        if sl is not None:
            add(x, "evade", sl)

    # R13: threats by a mover that stands on its destination
    if b1[to] == x:
        for y in neighbours(to):
            e = b1[y]
            if e >= 0 and owner(e) != me:
                sl = slot_seen(p1[e])
                if sl is not None:
                    add(x, "threat", sl)

    # R16: protection, a non-battle reply to a threat by A
    if A is not None and not battle and any(b0[y] >= 0 and owner(b0[y]) == me for y in neighbours(a)):
        for s in neighbours(a):
            if s in LAKES or s == frm or s in neighbours(frm) or s not in neighbours(to):
                continue
            occupant = b1[s]
            if occupant >= 0 and owner(occupant) == me:
                add(x, "prot", slot_guard(p1[occupant]))
                add(x, "prot_against", slot_guard(p1[A]))
                add(occupant, "been_by", slot_guard(p1[x]))
                add(occupant, "been_against", slot_guard(p1[A]))
            elif occupant == -1:
                add(x, "prot", 11)
                add(x, "prot_against", slot_guard(p1[A]))
    return inc


def check_games(n, seed, plies):
    eng = O.OracleEngine(n, seed, k_battleless=100, max_moves=1000, auto_reset=False)
    counts = dict.fromkeys(FIELDS, 0)
    checked = 0
    for _ in range(plies):
        pre = eng.export()
        r = eng.ply(obs=False, mask=False)
        post = eng.export()
        for g in range(n):
            if header(pre[g])["done"]:
                continue
            inc = expected_increments(pre[g], post[g], r["actions"][g])
            q0, q1 = unpack_pieces(pre[g]), unpack_pieces(post[g])
            for pid in range(80):
                for f in FIELDS:
                    want = q0[pid][f] | inc.get(pid, {}).get(f, 0)
                    assert q1[pid][f] == want, (
                        f"seed {seed} game {g} ply {header(pre[g])['ply']} action {r['actions'][g]}: "
                        f"piece {pid} {f} is {q1[pid][f]:#x}, the brute force gives {want:#x}")
                    if q1[pid][f] != q0[pid][f]:
                        counts[f] += 1
            checked += 1
    return counts, checked


def test_history_features_match_brute_force_every_ply():
    counts, checked = check_games(24, seed=11, plies=260)
    assert checked > 4000
    # every feature was exercised, not only compared as zero
    for f in FIELDS:
        assert counts[f] > 0, f"no ply ever set {f}"


def test_history_features_with_seed_variety():
    for seed in (3, 19):
        counts, checked = check_games(8, seed=seed, plies=200)
        assert checked > 1000
        assert counts["threat"] > 0 and counts["adj"] > 0


def check_position(rec, action):
    """One ply of a hand-built position against the brute force."""
    e = O.OracleEngine.from_records(np.stack([rec]), 1, k_battleless=100, max_moves=1000)
    e.step(np.array([action], dtype=np.int16))
    post = e.export()[0]
    inc = expected_increments(rec, post, action)
    q0, q1 = unpack_pieces(rec), unpack_pieces(post)
    for pid in range(80):
        for f in FIELDS:
            want = q0[pid][f] | inc.get(pid, {}).get(f, 0)
            assert q1[pid][f] == want, f"piece {pid} {f} is {q1[pid][f]:#x}, the brute force gives {want:#x}"
    return inc


def test_scout_passing_the_threatener_protects_nothing_it_already_touched():
    """Geometry random games almost never reach: blue's piece A has just
    stepped to (3,1), next to red's Sergeant at (3,0) (a threat), and red's
    Scout answers by running (2,0) -> (2,2) past it.  (2,1) is next to A and
    to the destination, but the Scout touched it before the move, so it is
    not newly guarded; (3,2), the other such square, holds a blue piece."""
    rec = make_record([dict(sq=sq(2, 0), owner=0, type="Scout"),
                       dict(sq=sq(3, 0), owner=0, type="Sergeant"),
                       dict(sq=sq(3, 1), owner=1, type="Captain", moved=1),
                       dict(sq=sq(3, 2), owner=1, type="Bomb"),
                       dict(sq=sq(0, 9), owner=0, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Flag")],
                      ply=2, moves=[(1, 11), (41, 31)])
    scout = board(rec)[sq(2, 0)]
    inc = check_position(rec, 100 * sq(2, 0) + sq(2, 2))
    assert "prot" not in inc.get(scout, {})
    # one square short, the Scout stops next to A: a threat on the hidden Captain
    inc = check_position(rec, 100 * sq(2, 0) + sq(2, 1))
    assert inc.get(scout, {}).get("threat") == 1 << 10      # next to the hidden Captain
