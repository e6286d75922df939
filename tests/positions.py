"""Hand-built game positions packed as canonical 1536-byte state records.

This module is an input generator shared by the oracle tests and the GPU
tests.  It only packs fields into the record layout; it holds none of the
engine's arithmetic (no move generation, battles, encoding or RNG).

Record layout (little-endian):
  0 u32 game_id | 4 u32 episode | 8 i32 ply | 12 i32 battleless
  16 u8 ring_count | 17 u8 done | 18 i8 outcome | 19 u8 reason | 20 u32 redraws
  24 + 8*p: two-square state of player p: u8 piece id | u8 n (0..4) | u8 squares[4]
  (the squares the piece occupied, oldest first, the last being its square)
  64..163 i8 board[100] (piece id, -1 empty, -2 lake)
  164..227 u8 ring[32][2] (from, to); the move made at ply t sits in slot t mod 32
  256 + 16*id: u32 w0, w1, w2, w3 per piece id (0..39 red, 40..79 blue)
    w0: type 0-3 | alive 4 | revealed 5 | moved 6 | death cause 7-9 |
        death square 10-16 (127 while alive) | been-protected-against 17-29 |
        long move 30 (the piece once moved more than one square)
    w1: threat 0-10 | evade 11-21
    w2: active adjacency 0-10 | protected 11-23
    w3: protected-against 0-12 | been-protected-by 13-25
"""
import numpy as np

TYPES = ["Spy", "Scout", "Miner", "Sergeant", "Lieutenant", "Captain", "Major", "Colonel",
         "General", "Marshal", "Flag", "Bomb"]
T = {name: i for i, name in enumerate(TYPES)}
COUNTS = [1, 8, 5, 4, 4, 4, 3, 2, 1, 1, 1, 6]
LAKES = {42, 43, 46, 47, 52, 53, 56, 57}
REC_BYTES = 1536

# default type of every piece id: the sorted multiset, per player
DEFAULT_TYPE = []
for _t, _c in enumerate(COUNTS):
    DEFAULT_TYPE += [_t] * _c
assert len(DEFAULT_TYPE) == 40


def start_square(pid):
    return pid if pid < 40 else 99 - (pid - 40)


def sq(row, col):
    return 10 * row + col


def make_record(pieces, ply=0, battleless=0, game_id=0, episode=0, moves=(), done=0,
                outcome=0, reason=0, dead_cause=6, dead_square=None, two_square=(None, None),
                dead=()):
    """pieces: list of dicts with keys sq, owner, type (name or index) and optional
    revealed, moved, long_move, id, threat, evade, adj, prot, prot_against, been_by,
    been_against.  Piece ids are taken from the owner's unused ids whose default
    type matches, unless `id` is given.
    dead: list of dicts with keys id, cause, sq (death square) and optional type
    (default: the id's default type): pieces captured with that cause on that square.
    Ids neither placed nor listed in `dead` become dead pieces too (revealed, death
    square = their start square unless dead_square is given, cause dead_cause).
    moves: list of (from, to), oldest first; stored as the last len(moves) plies
    before `ply`.
    two_square: per player None or a list of squares (oldest first) occupied by
    the piece that now stands on the last of them."""
    rec = np.zeros(REC_BYTES, dtype=np.uint8)
    board = np.full(100, -1, dtype=np.int8)
    for s in LAKES:
        board[s] = -2
    used = set()
    words = {}
    for p in pieces:
        t = p["type"] if isinstance(p["type"], int) else T[p["type"]]
        owner = p["owner"]
        pid = p.get("id")
        if pid is None:
            for cand in range(owner * 40, owner * 40 + 40):
                if cand not in used and DEFAULT_TYPE[cand - owner * 40] == t:
                    pid = cand
                    break
            if pid is None:
                for cand in range(owner * 40, owner * 40 + 40):
                    if cand not in used:
                        pid = cand
                        break
        assert pid not in used
        used.add(pid)
        s = p["sq"]
        assert s not in LAKES and board[s] == -1
        board[s] = pid
        w0 = t | (1 << 4) | (int(p.get("revealed", 0)) << 5) | (int(p.get("moved", 0)) << 6)
        w0 |= 127 << 10
        w0 |= int(p.get("long_move", 0)) << 30
        w0 |= int(p.get("been_against", 0)) << 17
        w1 = int(p.get("threat", 0)) | (int(p.get("evade", 0)) << 11)
        w2 = int(p.get("adj", 0)) | (int(p.get("prot", 0)) << 11)
        w3 = int(p.get("prot_against", 0)) | (int(p.get("been_by", 0)) << 13)
        words[pid] = (w0, w1, w2, w3)
    # explicitly captured pieces
    for d in dead:
        pid = d["id"]
        assert pid not in used
        used.add(pid)
        t = d.get("type", DEFAULT_TYPE[pid % 40])
        t = t if isinstance(t, int) else T[t]
        words[pid] = (t | (1 << 5) | (int(d["cause"]) << 7) | (int(d["sq"]) << 10), 0, 0, 0)
    # remaining ids are dead, with their default type unless already taken
    for owner in (0, 1):
        free_types = list(DEFAULT_TYPE)
        for pid in used:
            if pid // 40 == owner:
                free_types.remove(words[pid][0] & 15)
        for pid in range(owner * 40, owner * 40 + 40):
            if pid in used:
                continue
            t = free_types.pop(0)
            dsq = start_square(pid) if dead_square is None else dead_square
            w0 = t | (0 << 4) | (1 << 5) | (dead_cause << 7) | (dsq << 10)
            words[pid] = (w0, 0, 0, 0)
    def put32(off, v):
        rec[off:off + 4] = np.frombuffer(np.uint32(v & 0xFFFFFFFF).tobytes(), dtype=np.uint8)
    put32(0, game_id)
    put32(4, episode)
    put32(8, ply)
    put32(12, battleless)
    moves = list(moves)
    assert len(moves) <= 32 and len(moves) <= ply
    rec[16] = len(moves)
    rec[17] = done
    rec[18] = np.uint8(np.int8(outcome))
    rec[19] = reason
    rec[64:164] = board.view(np.uint8)
    for p, squares in enumerate(two_square):
        if squares:
            assert 2 <= len(squares) <= 4
            rec[24 + 8 * p] = board[squares[-1]]
            rec[25 + 8 * p] = len(squares)
            rec[26 + 8 * p:26 + 8 * p + len(squares)] = squares
    for i, (f, t_) in enumerate(moves):
        plyidx = ply - len(moves) + i
        slot = plyidx % 32
        rec[164 + 2 * slot] = f
        rec[165 + 2 * slot] = t_
    for pid, (w0, w1, w2, w3) in words.items():
        off = 256 + 16 * pid
        put32(off, w0)
        put32(off + 4, w1)
        put32(off + 8, w2)
        put32(off + 12, w3)
    return rec


def unpack_pieces(rec):
    """Decode the per-piece words of a record into a list of dicts (for checks)."""
    w = rec[256:256 + 1280].view(np.uint32).reshape(80, 4)
    out = []
    for pid in range(80):
        w0, w1, w2, w3 = (int(x) for x in w[pid])
        out.append(dict(
            id=pid, type=w0 & 15, alive=(w0 >> 4) & 1, revealed=(w0 >> 5) & 1,
            moved=(w0 >> 6) & 1, death_cause=(w0 >> 7) & 7, death_square=(w0 >> 10) & 127,
            been_against=(w0 >> 17) & 0x1FFF, long_move=(w0 >> 30) & 1,
            threat=w1 & 0x7FF, evade=(w1 >> 11) & 0x7FF, adj=w2 & 0x7FF, prot=(w2 >> 11) & 0x1FFF, prot_against=w3 & 0x1FFF,
            been_by=(w3 >> 13) & 0x1FFF))
    return out


def header(rec):
    h = rec[:24]
    return dict(game_id=int(h[0:4].view(np.uint32)[0]), episode=int(h[4:8].view(np.uint32)[0]),
                ply=int(h[8:12].view(np.int32)[0]), battleless=int(h[12:16].view(np.int32)[0]),
                ring_count=int(h[16]), done=int(h[17]), outcome=int(np.int8(h[18])),
                reason=int(h[19]), redraws=int(h[20:24].view(np.uint32)[0]))


def board(rec):
    return rec[64:164].view(np.int8).astype(int)
