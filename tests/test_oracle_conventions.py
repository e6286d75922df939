"""The random-number conventions of the oracle, recomputed independently (no GPU).

The paper names no generator; the readings fix one (Philox4x32-10, SC'11):
key = the 64-bit seed, counter = (game id, a, episode, tag), and
bounded(u, n) = (u * n) >> 32.  The generator itself is pinned by published
known-answer vectors elsewhere; here every decision built on it is recomputed
in plain Python from the stated conventions, for 1000 or more game ids, and
compared with what the oracle did:

* setups (tags 1 and 2): a Durstenfeld shuffle of the type multiset sorted in
  the channel order of App. C.1, i = 39 down to 1, j = bounded(next word, i+1),
  words x, y, z, w of blocks 0, 1, ... in turn; red id i on square i, blue id
  40 + i on square 99 - i;
* the uniform move (App. B SampleRandomLegalAction; tag 0, a = ply): the
  r-th legal action in ascending id order, r = bounded(word x, n);
* the magnet move (section 2.4: a piece with a legal move uniformly, then one
  of its moves; tag 0, a = ply): the r1-th such square ascending, r1 =
  bounded(word y, P), then its r2-th destination ascending, r2 =
  bounded(word z, m);
* the resample (section 2.5; tag 3, a = block, new game id): the Flag and the
  Bombs among the unmoved unknown pieces by a partial Fisher-Yates in
  ascending id order (position i takes j = i + bounded(next, nu - i); the
  first n_Flag chosen are Flags), then the movable multiset (sorted) shuffled
  by Durstenfeld and dealt to the remaining unknown pieces in ascending id order.
"""
import numpy as np

import oracle as O
from positions import COUNTS, T, header, unpack_pieces

SEED = 0x0123456789ABCDEF          # both key words differ from zero
FLAG, BOMB, SCOUT, MARSHAL = T["Flag"], T["Bomb"], T["Scout"], T["Marshal"]


def block(game_id, a, episode, tag, seed=SEED):
    key = [seed & 0xFFFFFFFF, seed >> 32]
    return [int(w) for w in O.philox4x32_10([game_id, a, episode, tag], key)]


def bounded(u, n):
    return (u * n) >> 32


class Words:
    """Words x, y, z, w of blocks 0, 1, 2, ... of one counter stream."""

    def __init__(self, game_id, episode, tag, seed=SEED):
        self.args = (game_id, episode, tag, seed)
        self.buf, self.block = [], 0

    def next(self):
        if not self.buf:
            g, ep, tag, seed = self.args
            self.buf = block(g, self.block, ep, tag, seed)
            self.block += 1
        return self.buf.pop(0)


SORTED = [t for t in range(12) for _ in range(COUNTS[t])]


def setup_types(game_id, episode, player):
    a = list(SORTED)
    ws = Words(game_id, episode, 1 + player)
    for i in range(39, 0, -1):
        j = bounded(ws.next(), i + 1)
        a[i], a[j] = a[j], a[i]
    return a


def test_setup_convention_for_1000_games():
    for g in range(1000):
        for p in (0, 1):
            assert list(O.setup_types(SEED, g, 0, p)) == setup_types(g, 0, p), (g, p)
    # the same types land on the stated squares of a fresh game record
    ids = np.arange(0, 3000, 50, dtype=np.uint32)
    e = O.OracleEngine(len(ids), SEED, game_ids=ids)
    for k, rec in enumerate(e.export()):
        pcs = unpack_pieces(rec)
        b = rec[64:164].view(np.int8)
        for p in (0, 1):
            types = setup_types(int(ids[k]), 0, p)
            for i in range(40):
                pid = 40 * p + i
                assert b[i if p == 0 else 99 - i] == pid
                assert pcs[pid]["type"] == types[i], (ids[k], p, i)


def legal_ids(mask_row):
    bits = np.unpackbits(mask_row.view(np.uint8), bitorder="little")
    return np.flatnonzero(bits).tolist()


def _games(n, plies, **kw):
    """n oracle games advanced some plies (the states the samplers act on)."""
    e = O.OracleEngine(n, SEED, auto_reset=True, **kw)
    for _ in range(plies):
        e.ply(obs=False, mask=False)
    return e


def test_uniform_move_convention_for_1000_games():
    e = _games(1000, 0)
    checked = 0
    for ply in range(24):
        mask, nl = e.mask()
        got = e.sample(mask, nl)
        for g, rec in enumerate(e.export()):
            h = header(rec)
            legal = legal_ids(mask[g])
            assert len(legal) == nl[g]
            if not legal:
                assert got[g] == -1
                continue
            x = block(h["game_id"], h["ply"], h["episode"], 0)[0]
            assert got[g] == legal[bounded(x, len(legal))], (g, ply)
            checked += 1
        e.step(got)
    assert checked >= 20000


def test_magnet_move_convention_for_1000_games():
    e = _games(1000, 0, sampler=O.SAMPLER_MAGNET)
    for ply in range(24):
        mask, nl = e.mask()
        got = e.sample(mask, nl)
        for g, rec in enumerate(e.export()):
            h = header(rec)
            legal = legal_ids(mask[g])
            if not legal:
                assert got[g] == -1
                continue
            by_square = {}
            for a in legal:                      # ascending ids: squares, then destinations
                by_square.setdefault(a // 100, []).append(a)
            squares = sorted(by_square)
            _, y, z, _ = block(h["game_id"], h["ply"], h["episode"], 0)
            moves = by_square[squares[bounded(y, len(squares))]]
            assert got[g] == moves[bounded(z, len(moves))], (g, ply)
        e.step(got)


def resample_types(src_rec, new_id):
    """The unknown types of the player not to move, redrawn by the convention."""
    h = header(src_rec)
    pcs = unpack_pieces(src_rec)
    z = 1 - (h["ply"] & 1)
    mine = pcs[40 * z:40 * z + 40]
    known = [p for p in mine if not p["alive"] or p["revealed"] or p["long_move"]]
    n = list(COUNTS)
    for p in known:
        n[p["type"]] -= 1
    unknown = [p["id"] for p in mine if p not in known]
    unmoved = [p["id"] for p in mine if p not in known and not p["moved"]]
    ws = Words(new_id, h["episode"], 3)
    I = n[FLAG] + n[BOMB]
    for i in range(I):
        j = i + bounded(ws.next(), len(unmoved) - i)
        unmoved[i], unmoved[j] = unmoved[j], unmoved[i]
    out = {pid: (FLAG if i < n[FLAG] else BOMB) for i, pid in enumerate(unmoved[:I])}
    movable = [t for t in range(MARSHAL + 1) for _ in range(n[t])]
    for i in range(len(movable) - 1, 0, -1):
        j = bounded(ws.next(), i + 1)
        movable[i], movable[j] = movable[j], movable[i]
    rest = [pid for pid in unknown if pid not in out]
    assert len(rest) == len(movable)
    out.update(zip(rest, movable))
    return out


def test_resample_convention_for_1024_resamples():
    e = _games(512, 90)
    recs = e.export()
    live = [g for g in range(512) if header(recs[g])["done"] == 0][:128]
    assert len(live) == 128
    src = O.OracleEngine.from_records(recs[live], SEED)
    per, base = 8, 5000
    out = src.resample(per, SEED, game_id_base=base).export()
    long_moves = 0
    for i, g in enumerate(live):
        long_moves += sum(p["long_move"] for p in unpack_pieces(recs[g]) if p["alive"])
        for j in range(per):
            k = i * per + j
            want = resample_types(recs[g], base + k)
            pcs = unpack_pieces(out[k])
            assert header(out[k])["game_id"] == base + k
            for pid, t in want.items():
                assert pcs[pid]["type"] == t, (g, j, pid)
            # everything else of the record is unchanged
            same = [p for p in range(80) if p not in want]
            src_pcs = unpack_pieces(recs[g])
            assert all(pcs[p] == src_pcs[p] for p in same)
    assert long_moves > 0          # the known-Scout case occurs in these states
