"""Pins of the rollout-buffer oracle (App. B.1), CPU only.

The defining property of the paper's rollout buffer is that a past mask or
information state recomputed from the recorded state equals the one the
simulator produced at that time step; the remaining queries are checked on
hand-built positions whose answers follow from the rules (App. A) and on
closed forms of the initial setup.
"""
import numpy as np
import pytest

from oracle import OracleEngine, OracleRolloutBuffer, WindowError
from positions import COUNTS, make_record, sq


def _run(n=16, plies=14, H=5, seed=11, auto_reset=True, k=100, max_moves=1000):
    e = OracleEngine(n, seed, k_battleless=k, max_moves=max_moves, auto_reset=auto_reset)
    buf = OracleRolloutBuffer(e, H)
    live = []
    for _ in range(plies):
        live.append(buf.ply(obs=True, mask=True))
    return buf, live


def test_window_and_ring():
    buf, _ = _run(plies=14, H=5)
    assert buf.window() == (9, 14)
    assert sorted(buf.rows) == [9, 10, 11, 12, 13]
    for t in (8, 15, -1):
        with pytest.raises(WindowError):
            buf.records_at(t)
    empty = OracleRolloutBuffer(OracleEngine(4, 1), 0)
    assert empty.window() == (0, 0)
    empty.ply(obs=False)
    assert empty.window() == (1, 1) and empty.rows == {}


def test_past_masks_and_obs_equal_those_produced_at_the_time():
    buf, live = _run(plies=14, H=5)
    lo, T = buf.window()
    for t in range(lo, T):
        m, nl = buf.mask_at(t)
        assert np.array_equal(m, live[t]["mask"])
        assert np.array_equal(nl, live[t]["num_legal"])
        assert np.array_equal(buf.obs_at(t), live[t]["obs"])
        info = buf.info_at(t)
        assert np.array_equal(info["played_action"], live[t]["actions"])
    # a subset with repeats, in any order
    games = [7, 0, 7, 15, 3]
    t = lo + 2
    m, _ = buf.mask_at(t, games)
    assert np.array_equal(m, live[t]["mask"][games])
    assert np.array_equal(buf.obs_at(t, games), live[t]["obs"][games])
    # the current step reads the live states
    m, nl = buf.mask_at(T)
    m2, nl2 = buf.e.mask()
    assert np.array_equal(m, m2) and np.array_equal(nl, nl2)
    assert (buf.info_at(T)["played_action"] == -1).all()


def test_rewind_from_a_past_record_replays_the_same_states():
    buf, live = _run(plies=12, H=8)
    lo, T = buf.window()
    t0 = lo + 1
    cfg = buf.e.cfg
    e = OracleEngine.from_records(buf.records_at(t0), cfg.seed, k_battleless=cfg.k_battleless,
                                  max_moves=cfg.max_moves, auto_reset=True)
    for t in range(t0, T):
        e.step(live[t]["actions"])
        assert np.array_equal(e.export(), buf.records_at(t + 1))


def test_scalars_follow_the_records():
    buf, live = _run(plies=12, H=6)
    lo, T = buf.window()
    for t in range(lo, T + 1):
        info = buf.info_at(t)
        rec = buf.records_at(t)
        ply = rec[:, 8:12].copy().view(np.uint32)[:, 0]
        assert np.array_equal(info["acting_player"], (ply & 1).astype(np.int8))
        assert np.array_equal(info["num_moves"], ply.astype(np.int32))
        assert np.array_equal(info["moves_since_attack"], rec[:, 12:16].copy().view(np.uint32)[:, 0])
        _, nl = buf.mask_at(t)
        assert np.array_equal(info["has_legal_movement"], (nl > 0).astype(np.uint8))
        if t < T:
            ended = live[t]["done"].astype(bool)   # auto-reset: every done is an episode end
            assert np.array_equal(info["reward_pl0"], np.where(ended, live[t]["outcome"], 0))
            assert np.array_equal(info["flag_captured"], (ended & (live[t]["reason"] == 1)).astype(np.uint8))
        assert (info["terminated_since"] == 0).all()


def _flag_position(mover):
    """mover's Sergeant next to the opponent's Flag; both sides keep a Scout."""
    if mover == 0:
        pieces = [dict(sq=sq(6, 5), owner=0, type="Sergeant"), dict(sq=sq(0, 0), owner=0, type="Scout"),
                  dict(sq=sq(7, 5), owner=1, type="Flag"), dict(sq=sq(9, 9), owner=1, type="Scout")]
        return make_record(pieces, ply=0), 100 * sq(6, 5) + sq(7, 5)
    pieces = [dict(sq=sq(3, 4), owner=1, type="Sergeant"), dict(sq=sq(9, 9), owner=1, type="Scout"),
              dict(sq=sq(2, 4), owner=0, type="Flag"), dict(sq=sq(0, 0), owner=0, type="Scout")]
    return make_record(pieces, ply=1, moves=[(sq(0, 1), sq(0, 0))]), 100 * sq(3, 4) + sq(2, 4)


@pytest.mark.parametrize("mover,reward", [(0, 1), (1, -1)])
def test_flag_capture_reward_and_terminated_since(mover, reward):
    rec, action = _flag_position(mover)
    e = OracleEngine.from_records(rec[None], seed=3, auto_reset=False)
    buf = OracleRolloutBuffer(e, 8)
    buf.step(np.array([action], np.int16))
    for _ in range(3):
        buf.step(np.array([-1], np.int16))
    i0 = buf.info_at(0)
    assert i0["acting_player"][0] == mover
    assert i0["played_action"][0] == action
    assert i0["reward_pl0"][0] == reward and i0["flag_captured"][0] == 1
    assert i0["terminated_since"][0] == 0 and i0["has_legal_movement"][0] == 1
    for t in (1, 2, 3, 4):
        it = buf.info_at(t)
        assert it["terminated_since"][0] == t
        assert it["reward_pl0"][0] == 0 and it["flag_captured"][0] == 0
        assert it["has_legal_movement"][0] == 0
    m, nl = buf.mask_at(2)
    assert nl[0] == 0 and not m.any()
    # a short window only sees part of the terminal run
    short = OracleRolloutBuffer(OracleEngine.from_records(rec[None], seed=3, auto_reset=False), 2)
    short.step(np.array([action], np.int16))
    for _ in range(3):
        short.step(np.array([-1], np.int16))
    assert short.window() == (2, 4)
    assert short.info_at(4)["terminated_since"][0] == 3


def test_piece_views_of_fresh_setups():
    e = OracleEngine(6, seed=21)
    buf = OracleRolloutBuffer(e, 2)
    buf.ply(obs=False)
    for t in (0, 1):
        info = buf.info_at(t)
        p = info["acting_player"]
        assert list(p) == [t] * 6
        oh = info["piece_onehot"]
        # own and opposing counts are the initial multiset (a Scout's first
        # move may already capture, so after one ply they can only be lower)
        full = np.tile(COUNTS, (6, 1))
        own_counts, opp_counts = oh[:, :12].sum(axis=2), oh[:, 12:].sum(axis=2)
        if t == 0:
            assert np.array_equal(own_counts, full) and np.array_equal(opp_counts, full)
        else:
            assert (own_counts <= full).all() and (opp_counts <= full).all()
            assert (own_counts.sum(axis=1) >= 39).all() and (opp_counts.sum(axis=1) >= 39).all()
        assert oh.sum(axis=1).max() == 1
        # the acting player's own pieces stand in the first four rows of its own frame
        own = oh[:, :12].sum(axis=1)
        assert (own[:, 40:] == 0).all()
        if t == 0:
            assert (own[:, :40] == 1).all()
            # nothing is revealed before the first battle: all 40 opposing pieces are unknown
            assert (info["is_unknown"].sum(axis=1) == 40).all()
            assert (info["is_unknown"][:, 60:] == 1).all()


def test_revealed_opponent_piece_is_known():
    pieces = [dict(sq=sq(3, 3), owner=0, type="Captain"), dict(sq=sq(6, 3), owner=1, type="Major",
                                                               revealed=1),
              dict(sq=sq(6, 6), owner=1, type="Bomb"), dict(sq=sq(9, 0), owner=1, type="Scout")]
    rec = make_record(pieces, ply=0)
    buf = OracleRolloutBuffer(OracleEngine.from_records(rec[None], seed=1), 1)
    info = buf.info_at(0)
    assert info["is_unknown"][0, sq(6, 3)] == 0
    assert info["is_unknown"][0, sq(6, 6)] == 1 and info["is_unknown"][0, sq(9, 0)] == 1
    assert info["is_unknown"][0].sum() == 2
    oh = info["piece_onehot"][0]
    assert oh[12 + 6, sq(6, 3)] == 1 and oh[12 + 11, sq(6, 6)] == 1 and oh[5, sq(3, 3)] == 1
    # blue to move sees the board rotated by 180 degrees
    rec_b = make_record(pieces, ply=1, moves=[(sq(3, 2), sq(3, 3))])
    info_b = OracleRolloutBuffer(OracleEngine.from_records(rec_b[None], seed=1), 1).info_at(0)
    oh_b = info_b["piece_onehot"][0]
    assert oh_b[6, 99 - sq(6, 3)] == 1 and oh_b[12 + 5, 99 - sq(3, 3)] == 1
    assert info_b["is_unknown"][0].sum() == 1 and info_b["is_unknown"][0, 99 - sq(3, 3)] == 1
