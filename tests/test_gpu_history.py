"""Rollout buffer (App. B.1) on the GPU vs the oracle's, bit-exact: masks,
information states, records and the scalar/per-square queries at every time
step of the window, after fused plies (with and without observations, direct
and replayed from graphs) and plain steps."""
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


def compare_window(eng, buf, games_list=None, obs=True):
    lo, T = buf.window()
    assert eng.window() == (lo, T)
    for t in range(lo, T + 1):
        for games in (None, games_list):
            g_dev = None if games is None else torch.tensor(games, dtype=torch.int32, device="cuda")
            tag = f"t={t} {'all' if games is None else 'list'}"
            m, nl = eng.mask_at(t, g_dev)
            wm, wnl = buf.mask_at(t, games)
            assert_same(f"mask {tag}", cpu(m), wm)
            assert_same(f"num_legal {tag}", cpu(nl), wnl)
            assert_same(f"records {tag}", cpu(eng.export_at(t, g_dev)), buf.records_at(t, games))
            info = eng.info_at(t, g_dev)
            want = buf.info_at(t, games)
            for k, v in want.items():
                assert_same(f"{k} {tag}", cpu(info[k]), v)
            if obs:
                assert_same(f"obs {tag}", cpu(eng.obs_at(t, g_dev)), buf.obs_at(t, games))
    assert eng.error() == (0, -1)


def test_fused_plies_direct_and_from_graphs():
    """300 games (ragged against four-wave workgroups), ring of 6 steps, short
    episodes so that ends, resets and flag captures fall inside the window.
    Plies alternate between single launches with observations and replays of
    a captured 3-ply graph without them."""
    n, seed, H = 300, 17, 6
    kw = dict(k_battleless=12, max_moves=60, auto_reset=True)
    eng = E.Engine(n, seed, history_len=H, **kw)
    buf = O.OracleRolloutBuffer(O.OracleEngine(n, seed, **kw), H)
    rng = np.random.default_rng(0)
    games = [int(x) for x in rng.integers(0, n, 77)] + [0, n - 1, 5, 5]
    acts = torch.empty((3, n), dtype=torch.int16, device="cuda")
    for rnd in range(6):
        E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, num_legal=eng.num_legal, actions=eng.actions,
                             obs=eng.obs, done=eng.done, outcome=eng.outcome, reason=eng.reason,
                             ep_len=eng.ep_len)
        r = buf.ply(obs=True)
        assert_same(f"actions@{rnd}", cpu(eng.actions), r["actions"])
        assert_same(f"obs@{rnd}", cpu(eng.obs), r["obs"])
        # the same graph replayed every round: each replay must take fresh ring rows
        E.stratego_run_plies(eng.ctx, 3, actions=acts, use_graph=True)
        for p in range(3):
            r = buf.ply(obs=False)
            assert_same(f"graph actions@{rnd}.{p}", cpu(acts[p]), r["actions"])
        if rnd in (1, 5):
            compare_window(eng, buf, games, obs=rnd == 5)
    assert eng.window() == (24 - H, 24)
    eng.close()


def test_plain_steps_without_auto_reset():
    """stratego_step records too; finished games stay finished, so the
    terminated-since counts and episode-ending rewards show up."""
    n, seed, H = 96, 5, 7
    kw = dict(k_battleless=10, max_moves=24, auto_reset=False)
    eng = E.Engine(n, seed, history_len=H, **kw)
    ref = O.OracleEngine(n, seed, **kw)
    buf = O.OracleRolloutBuffer(ref, H)
    for ply in range(30):
        eng.legal_mask()
        eng.sample()
        eng.step()
        m, nl = ref.mask()
        a = ref.sample(m, nl)
        buf.step(a)
        assert_same(f"actions@{ply}", cpu(eng.actions), a)
    info = buf.info_at(buf.window()[1])
    assert info["terminated_since"].max() >= H   # the run reaches past the window
    compare_window(eng, buf, [3, 1, 4, 1, 5, 9, 2, 6, 95], obs=True)
    eng.close()


def test_rewind_to_a_past_step_replays_it():
    n, seed, H = 128, 9, 5
    eng = E.Engine(n, seed, history_len=H, auto_reset=True)
    acts = torch.empty((4, n), dtype=torch.int16, device="cuda")
    E.stratego_run_plies(eng.ctx, 4, actions=acts)
    t0 = 1
    past = eng.export_at(t0)
    later = eng.export_at(4)
    eng.load(past)                       # every game back to time step 1
    E.stratego_run_plies(eng.ctx, 3, actions=acts[:3])
    assert torch.equal(eng.export(), later)
    # the rewound plies are new time steps in the ring
    assert eng.window() == (2, 7)
    assert torch.equal(eng.export_at(4), past)
    eng.close()


def test_window_and_argument_errors():
    n = 64
    eng = E.Engine(n, 2, history_len=3, auto_reset=True)
    assert eng.window() == (0, 0)
    E.stratego_run_plies(eng.ctx, 5)
    assert eng.window() == (2, 5)
    for t in (1, 6, -1):
        with pytest.raises(E.StrategoError) as err:
            eng.mask_at(t)
        assert err.value.code == E.E_RANGE
    slots = torch.arange(4, dtype=torch.int32, device="cuda")
    with pytest.raises(E.StrategoError) as err:
        E.stratego_run_plies_slots(eng.ctx, slots, 1)
    assert err.value.code == E.E_INVAL
    recs = eng.export()
    with pytest.raises(E.StrategoError) as err:
        E.stratego_serve(eng.ctx, [(E.REQ_ROLLOUT, 2, 4, 0, 0.0)], recs, recs.clone())
    assert err.value.code == E.E_INVAL
    # an index outside [0, N) is skipped and latched with its list position
    bad = torch.tensor([0, 7, n, 3], dtype=torch.int32, device="cuda")
    eng.mask_at(4, bad)
    assert eng.error() == (E.E_BAD_STATE, 2)
    # empty queries are no-ops
    eng.mask_at(4, torch.empty(0, dtype=torch.int32, device="cuda"))
    assert eng.error() == (0, -1)
    eng.close()
    # without a ring only the current step can be queried
    eng = E.Engine(n, 2, history_len=0)
    E.stratego_run_plies(eng.ctx, 2)
    assert eng.window() == (2, 2)
    with pytest.raises(E.StrategoError):
        eng.obs_at(1)
    ref = O.OracleEngine(n, 2)
    ref.ply(obs=False)
    ref.ply(obs=False)
    assert_same("obs at T", cpu(eng.obs_at(2)), ref.encode())
    eng.close()


def test_flag_capture_queries():
    """Hand-built: red captures the Flag at step 0, blue at step 0 of a second
    game; then both stay finished (no auto-reset)."""
    red = [dict(sq=sq(6, 5), owner=0, type="Sergeant"), dict(sq=sq(0, 0), owner=0, type="Scout"),
           dict(sq=sq(7, 5), owner=1, type="Flag"), dict(sq=sq(9, 9), owner=1, type="Scout")]
    blue = [dict(sq=sq(3, 4), owner=1, type="Sergeant"), dict(sq=sq(9, 9), owner=1, type="Scout"),
            dict(sq=sq(2, 4), owner=0, type="Flag"), dict(sq=sq(0, 0), owner=0, type="Scout")]
    recs = np.stack([make_record(red, ply=0), make_record(blue, ply=1, moves=[(sq(0, 1), sq(0, 0))])])
    actions = np.array([100 * sq(6, 5) + sq(7, 5), 100 * sq(3, 4) + sq(2, 4)], np.int16)
    eng = E.Engine(2, 3, history_len=4, auto_reset=False)
    eng.load(torch.from_numpy(recs).cuda())
    buf = O.OracleRolloutBuffer(O.OracleEngine.from_records(recs, 3, auto_reset=False), 4)
    for a in (actions, np.array([-1, -1], np.int16), np.array([-1, -1], np.int16)):
        E.stratego_step(eng.ctx, torch.from_numpy(a).cuda())
        buf.step(a)
    i0 = eng.info_at(0)
    assert cpu(i0["reward_pl0"]).tolist() == [1, -1]
    assert cpu(i0["flag_captured"]).tolist() == [1, 1]
    assert cpu(eng.info_at(3)["terminated_since"]).tolist() == [3, 3]
    compare_window(eng, buf, [1, 0, 1], obs=True)
    eng.close()


def test_65536_games_ring_against_live_outputs_and_sampled_oracle():
    """The bench configuration with a ring of 8: masks at every past step
    equal those the plies produced; observations at the last step equal the
    last ply's; 256 sampled games per step against the oracle."""
    n, seed, H = 65536, 1, 8
    eng = E.Engine(n, seed, k_battleless=100, max_moves=1000, auto_reset=True, history_len=H)
    E.stratego_run_plies(eng.ctx, 64, use_graph=True)          # desynchronise
    masks = []
    for _ in range(H):
        E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, num_legal=eng.num_legal, obs=eng.obs)
        masks.append((eng.mask.clone(), eng.num_legal.clone()))
    lo, T = eng.window()
    assert (lo, T) == (64, 72)
    for t in range(lo, T):
        m, nl = eng.mask_at(t)
        assert torch.equal(m, masks[t - lo][0]) and torch.equal(nl, masks[t - lo][1]), t
    assert torch.equal(eng.obs_at(T - 1), eng.obs)
    rng = np.random.default_rng(3)
    for t in (lo, T - 1, T):
        ids = np.sort(rng.choice(n, 256, replace=False)).astype(np.int32)
        g = torch.from_numpy(ids).cuda()
        rec = cpu(eng.export_at(t, g))
        ref = O.OracleEngine.from_records(rec, seed, k_battleless=100, max_moves=1000, auto_reset=True)
        wm, wnl = ref.mask()
        m, nl = eng.mask_at(t, g)
        assert_same(f"mask t={t}", cpu(m), wm)
        assert_same(f"obs t={t}", cpu(eng.obs_at(t, g)), ref.encode())
    assert eng.error() == (0, -1)
    eng.close()


def test_acting_player_views_at_past_steps():
    """With acting_obs_only the ring re-materialises the acting player's view
    ([count, 1, 488, 10, 10]) at every step of the window, equal to the live
    outputs of the plies and to the oracle's."""
    n, seed, H = 200, 8, 5
    kw = dict(k_battleless=15, max_moves=80, auto_reset=True)
    eng = E.Engine(n, seed, history_len=H, acting_obs=True, **kw)
    buf = O.OracleRolloutBuffer(O.OracleEngine(n, seed, acting_obs=True, **kw), H)
    live = []
    for ply in range(7):
        E.stratego_run_plies(eng.ctx, 1, obs=eng.obs)
        r = buf.ply(obs=True)
        assert_same(f"obs@{ply}", cpu(eng.obs), r["obs"])
        live.append(eng.obs.clone())
    lo, T = eng.window()
    assert (lo, T) == (2, 7)
    games = [0, 199, 17, 17, 100]
    g_dev = torch.tensor(games, dtype=torch.int32, device="cuda")
    for t in range(lo, T + 1):
        got = eng.obs_at(t)
        assert got.shape == (n, 1, 488, 10, 10)
        assert_same(f"obs at {t}", cpu(got), buf.obs_at(t))
        assert_same(f"obs at {t} (list)", cpu(eng.obs_at(t, g_dev)), buf.obs_at(t, games))
        if t < T:
            assert torch.equal(got, live[t])
    assert eng.error() == (0, -1)
    eng.close()


def test_board_strings_match_the_oracle():
    """BoardStrs (App. B): the library's text pictures at every step of the
    window and for all games now equal the oracle's; errors for a step
    outside the window and an index outside the games."""
    n, seed, H = 50, 4, 3
    kw = dict(k_battleless=20, max_moves=100, auto_reset=True)
    eng = E.Engine(n, seed, history_len=H, **kw)
    ref = O.OracleEngine(n, seed, **kw)
    buf = O.OracleRolloutBuffer(ref, H)
    for _ in range(5):
        E.stratego_run_plies(eng.ctx, 1)
        buf.ply(obs=False, mask=False)
    lo, T = eng.window()
    games = [0, 49, 7, 7]
    g_dev = torch.tensor(games, dtype=torch.int32, device="cuda")
    for t in range(lo, T + 1):
        at = O.OracleEngine.from_records(buf.records_at(t, games), seed, **kw)
        assert eng.board_strs(t, g_dev) == [at.board_string(i) for i in range(len(games))], t
    now = eng.board_strs()
    assert now == [ref.board_string(g) for g in range(n)]
    assert all(len(s.splitlines()) == 10 for s in now)
    with pytest.raises(E.StrategoError) as err:
        eng.board_strs(lo - 1)
    assert err.value.code == E.E_RANGE
    with pytest.raises(E.StrategoError) as err:
        eng.board_strs(T, torch.tensor([3, n], dtype=torch.int32, device="cuda"))
    assert err.value.code == E.E_INVAL
    eng.close()
