"""The competitive-play rules (App. A) on the GPU vs the oracle, bit-exact:
the two-square rule (App. B.2) and the continuous-chasing rule (Table
"chase", App. B.3) in masks, sampled and caller actions, outcomes, records
(which carry both rules' state) and the rule-applies queries."""
import numpy as np
import pytest

import oracle as O
from positions import make_record, sq

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2511_07312_amd import engine as E  # noqa: E402


def cpu(t):
    a = t.cpu().numpy()
    return a.view(np.uint64) if a.dtype == np.int64 and a.ndim == 2 and a.shape[-1] == 157 else a


def assert_same(name, got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (name, got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{name}: {len(bad)} mismatches, first at {bad[:5].tolist()}")


def sparse_positions(count, seed):
    from test_oracle_pins import random_position
    rng = np.random.default_rng(seed)
    return np.stack([random_position(rng, int(rng.integers(1, 7)), int(rng.integers(1, 7)))
                     for _ in range(count)])


@pytest.mark.parametrize("G,L", [(1, 1), (4, 3)])
def test_fused_plies_with_the_rule_in_sparse_positions(G, L):
    """Few pieces per side, so pieces shuttle and the rule bites often."""
    recs = sparse_positions(2000, seed=G)
    n, seed = len(recs), 7
    kw = dict(k_battleless=100, max_moves=300, auto_reset=False)
    eng = E.Engine(n, seed, two_square=True, games_per_wg=G, lds_layout=L, **kw)
    eng.load(torch.from_numpy(recs).cuda())
    assert eng.error() == (0, -1)
    ref = O.OracleEngine.from_records(recs, seed, two_square=True, **kw)
    applies = torch.empty(n, dtype=torch.uint8, device="cuda")
    bit = 0
    for ply in range(150):
        E.stratego_history_info(eng.ctx, eng.window()[1], None, n, two_square_applies=applies)
        want = np.array([ref.two_square_applies(g) for g in range(n)], dtype=np.uint8)
        assert_same(f"applies@{ply}", cpu(applies), want)
        bit += int(want.sum())
        obs = ply % 25 == 0
        E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, num_legal=eng.num_legal, actions=eng.actions,
                             obs=eng.obs if obs else None, done=eng.done, outcome=eng.outcome,
                             reason=eng.reason, ep_len=eng.ep_len)
        r = ref.ply(obs=obs)
        assert_same(f"mask@{ply}", cpu(eng.mask), r["mask"])
        assert_same(f"actions@{ply}", cpu(eng.actions), r["actions"])
        if obs:
            assert_same(f"obs@{ply}", cpu(eng.obs), r["obs"])
        for k in ("done", "outcome", "reason", "ep_len"):
            assert_same(f"{k}@{ply}", cpu(getattr(eng, k)), r[k])
        assert_same(f"states@{ply}", cpu(eng.export()), ref.export())
    assert bit > 200, bit        # the rule removed moves in many (game, ply) pairs
    assert eng.error() == (0, -1)
    eng.close()


def test_rule_off_matches_the_oracle():
    recs = sparse_positions(500, seed=3)
    n, seed = len(recs), 2
    eng = E.Engine(n, seed, max_moves=300, two_square=False)
    eng.load(torch.from_numpy(recs).cuda())
    ref = O.OracleEngine.from_records(recs, seed, max_moves=300, two_square=False)
    for ply in range(60):
        E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, actions=eng.actions)
        r = ref.ply(obs=False)
        assert_same(f"mask@{ply}", cpu(eng.mask), r["mask"])
    assert_same("states", cpu(eng.export()), ref.export())
    eng.close()


def test_caller_actions_forbidden_by_the_rule_are_rejected():
    A, B = sq(3, 0), sq(4, 0)
    rec = make_record([dict(sq=A, owner=0, type="Sergeant"), dict(sq=sq(0, 9), owner=0, type="Flag"),
                       dict(sq=sq(9, 9), owner=1, type="Scout"), dict(sq=sq(9, 0), owner=1, type="Flag")])
    seq = [100 * A + B, 9998, 100 * B + A, 9899, 100 * A + B, 9998]
    eng = E.Engine(1, 1, two_square=True, history_len=8)
    eng.load(torch.from_numpy(rec[None]).cuda())
    ref = O.OracleEngine.from_records(rec[None], 1, two_square=True)
    for a in seq:
        E.stratego_step(eng.ctx, torch.tensor([a], dtype=torch.int16, device="cuda"))
        ref.step(np.array([a], np.int16))
        eng.legal_mask()
        m, nl = ref.mask()
        assert_same(f"mask after {a}", cpu(eng.mask), m)
    assert_same("state", cpu(eng.export()), ref.export())
    info = eng.info_at(eng.window()[1])
    assert int(info["two_square_applies"][0]) == 1
    before = eng.export()
    E.stratego_step(eng.ctx, torch.tensor([100 * B + A], dtype=torch.int16, device="cuda"))
    assert eng.error() == (E.E_ILLEGAL_ACTION, 0)
    assert torch.equal(eng.export(), before)
    # an imported record with a malformed rule state is refused
    bad = rec.copy()
    bad[25] = 5
    eng.load(torch.from_numpy(bad[None]).cuda())
    assert eng.error() == (E.E_BAD_STATE, 0)
    eng.close()


def test_dead_end_loss_matches_the_oracle():
    walls = [dict(sq=s, owner=0, type="Bomb") for s in (sq(0, 1), sq(1, 1), sq(2, 0))]
    pieces = [dict(sq=sq(0, 0), owner=0, type="Sergeant"), dict(sq=sq(0, 9), owner=0, type="Flag")] + walls + [
        dict(sq=sq(9, 9), owner=1, type="Scout"), dict(sq=sq(9, 0), owner=1, type="Flag")]
    rec = make_record(pieces)
    seq = [100 * 0 + 10, 9998, 100 * 10 + 0, 9899, 100 * 0 + 10, 9998]
    for rule in (True, False):
        eng = E.Engine(1, 1, two_square=rule)
        eng.load(torch.from_numpy(rec[None]).cuda())
        ref = O.OracleEngine.from_records(rec[None], 1, two_square=rule)
        for a in seq:
            eng.step(torch.tensor([a], dtype=torch.int16, device="cuda"))
            r = ref.step(np.array([a], np.int16))
        for k in ("done", "outcome", "reason"):
            assert_same(k, cpu(getattr(eng, k)), r[k])
        assert int(eng.done[0]) == (1 if rule else 0)
        assert eng.error() == (0, -1)
        eng.close()


# ---------------------------------------------------------------- continuous-chasing rule
def test_chase_driven_games_match_the_oracle():
    """Sparse games whose moves keep chases going (threats first, then
    evasions): chase state, masks, outcomes and records bit-exact, the
    caller actions validated by the kernels, the rule biting many times."""
    from test_oracle_pins import chasing_actions, random_position
    rng = np.random.default_rng(23)
    recs = np.stack([random_position(rng, int(rng.integers(1, 4)), int(rng.integers(1, 4)))
                     for _ in range(400)])
    n, seed = len(recs), 4
    kw = dict(k_battleless=100, max_moves=400, auto_reset=False, chasing=True)
    eng = E.Engine(n, seed, **kw)
    eng.load(torch.from_numpy(recs).cuda())
    ref = O.OracleEngine.from_records(recs, seed, **kw)
    applies = torch.empty(n, dtype=torch.uint8, device="cuda")
    bites = 0
    for ply in range(100):
        E.stratego_history_info(eng.ctx, eng.window()[1], None, n, chase_applies=applies)
        want = np.array([ref.chase_applies(g) for g in range(n)], dtype=np.uint8)
        assert_same(f"chase applies@{ply}", cpu(applies), want)
        bites += int(want.sum())
        eng.legal_mask()
        m, nl = ref.mask()
        assert_same(f"mask@{ply}", cpu(eng.mask), m)
        a = chasing_actions(ref, rng)
        r = ref.step(a)
        eng.step(torch.from_numpy(a).cuda())
        for k in ("done", "outcome", "reason", "ep_len"):
            assert_same(f"{k}@{ply}", cpu(getattr(eng, k)), r[k])
        assert_same(f"states@{ply}", cpu(eng.export()), ref.export())
    assert bites >= 50, bites
    assert eng.error() == (0, -1)
    eng.close()


def test_chase_scenario_and_forbidden_caller_action():
    from test_oracle_pins import _CHASE, _chase_position
    rec = _chase_position()
    eng = E.Engine(1, 1, chasing=True)
    eng.load(torch.from_numpy(rec[None]).cuda())
    for a in _CHASE:
        E.stratego_step(eng.ctx, torch.tensor([a], dtype=torch.int16, device="cuda"))
    assert eng.error() == (0, -1)
    st = cpu(eng.export())[0]
    assert int(st[40]) == 8 and int(st[41]) == 0
    eng.legal_mask()
    m = cpu(eng.mask)[0]
    bit = lambda act: (int(m[act >> 6]) >> (act & 63)) & 1
    assert bit(212) == 0 and bit(203) == 1
    before = eng.export()
    E.stratego_step(eng.ctx, torch.tensor([212], dtype=torch.int16, device="cuda"))
    assert eng.error() == (E.E_ILLEGAL_ACTION, 0)
    assert torch.equal(eng.export(), before)
    eng.close()


@pytest.mark.parametrize("G,L", [(1, 1), (2, 4)])
def test_fused_plies_with_both_rules(G, L):
    recs = sparse_positions(1500, seed=11 + G)
    n, seed = len(recs), 9
    kw = dict(k_battleless=100, max_moves=300, auto_reset=False, two_square=True, chasing=True)
    eng = E.Engine(n, seed, games_per_wg=G, lds_layout=L, **kw)
    eng.load(torch.from_numpy(recs).cuda())
    ref = O.OracleEngine.from_records(recs, seed, **kw)
    for ply in range(120):
        obs = ply % 40 == 0
        E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, actions=eng.actions, obs=eng.obs if obs else None,
                             done=eng.done, outcome=eng.outcome, reason=eng.reason)
        r = ref.ply(obs=obs)
        assert_same(f"mask@{ply}", cpu(eng.mask), r["mask"])
        assert_same(f"actions@{ply}", cpu(eng.actions), r["actions"])
        if obs:
            assert_same(f"obs@{ply}", cpu(eng.obs), r["obs"])
        for k in ("done", "outcome", "reason"):
            assert_same(f"{k}@{ply}", cpu(getattr(eng, k)), r[k])
    assert_same("states", cpu(eng.export()), ref.export())
    assert eng.error() == (0, -1)
    eng.close()
