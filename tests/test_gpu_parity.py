"""GPU engine vs CPU oracle, bit-exact (integer work: states, masks, actions,
observations and outcomes must be identical)."""
import numpy as np
import pytest

import oracle as O
from digest import DeviceDigest
from positions import header, make_record, sq

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


# ---------------------------------------------------------------- plain engine
def test_plain_engine_256_games_200_plies():
    """Plain per-step kernels: 256 games, 200 plies, no auto-reset; every mask,
    action, observation, step output and state compared every ply."""
    n, seed = 256, 1
    eng = E.Engine(n, seed, k_battleless=100, max_moves=1000)
    ref = O.OracleEngine(n, seed, k_battleless=100, max_moves=1000)
    assert_same("initial states", cpu(eng.export()), ref.export())
    for ply in range(200):
        eng.legal_mask()
        eng.sample()
        eng.encode()
        eng.step()
        m, nl = ref.mask()
        a = ref.sample(m, nl)
        obs = ref.encode()
        r = ref.step(a)
        assert_same(f"mask@{ply}", cpu(eng.mask), m)
        assert_same(f"num_legal@{ply}", cpu(eng.num_legal), nl)
        assert_same(f"actions@{ply}", cpu(eng.actions), a)
        assert_same(f"obs@{ply}", cpu(eng.obs), obs)
        for k in ("done", "outcome", "reason", "ep_len"):
            assert_same(f"{k}@{ply}", cpu(getattr(eng, k)), r[k])
        assert_same(f"states@{ply}", cpu(eng.export()), ref.export())
    assert eng.error() == (0, -1)
    eng.close()


# ---------------------------------------------------------------- fused engine
# (games per workgroup, LDS layout): layout 1 = bit planes, 2..6 = byte images
# in 1, 2, 4, 8, 16 channel segments, 7 = bit planes of one observer at a time
TILINGS = [(1, 1), (2, 1), (4, 1), (8, 1), (16, 1), (1, 2), (2, 3), (4, 4), (8, 5), (16, 6), (1, 7), (4, 7)]


@pytest.mark.parametrize("G,L", TILINGS)
def test_fused_engine_every_tiling(G, L):
    """Fused persistent kernel, auto-reset on: per ply mask, actions, obs, step
    outputs and states equal the oracle for every (games per WG, LDS layout)."""
    n, seed, plies = 1000, 3, 40 if (G, L) != (1, 1) else 160
    eng = E.Engine(n, seed, k_battleless=100, max_moves=1000, auto_reset=True,
                   games_per_wg=G, lds_layout=L)
    ref = O.OracleEngine(n, seed, k_battleless=100, max_moves=1000, auto_reset=True)
    for ply in range(plies):
        E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, num_legal=eng.num_legal,
                             actions=eng.actions, obs=eng.obs, done=eng.done, outcome=eng.outcome,
                             reason=eng.reason, ep_len=eng.ep_len)
        r = ref.ply(obs=True)
        assert_same(f"mask@{ply}", cpu(eng.mask), r["mask"])
        assert_same(f"num_legal@{ply}", cpu(eng.num_legal), r["num_legal"])
        assert_same(f"actions@{ply}", cpu(eng.actions), r["actions"])
        assert_same(f"obs@{ply}", cpu(eng.obs), r["obs"])
        for k in ("done", "outcome", "reason", "ep_len"):
            assert_same(f"{k}@{ply}", cpu(getattr(eng, k)), r[k])
        assert_same(f"states@{ply}", cpu(eng.export()), ref.export())
    eng.close()


def test_graph_64_plies_auto_reset():
    """One hipGraph of 64 fused plies (twice): per-ply outputs and final states."""
    n, seed, P = 4096, 5, 64
    eng = E.Engine(n, seed, k_battleless=100, max_moves=1000, auto_reset=True)
    ref = O.OracleEngine(n, seed, k_battleless=100, max_moves=1000, auto_reset=True)
    acts = torch.empty((P, n), dtype=torch.int16, device="cuda")
    done = torch.empty((P, n), dtype=torch.int8, device="cuda")
    outc = torch.empty((P, n), dtype=torch.int8, device="cuda")
    reas = torch.empty((P, n), dtype=torch.uint8, device="cuda")
    epl = torch.empty((P, n), dtype=torch.int16, device="cuda")
    ns = torch.empty(P, dtype=torch.int64, device="cuda")
    for rep in range(2):
        E.stratego_run_plies(eng.ctx, P, mask=eng.mask, actions=acts, obs=eng.obs, done=done,
                             outcome=outc, reason=reas, ep_len=epl, use_graph=True, ply_ns=ns)
        for p in range(P):
            r = ref.ply(obs=(p == P - 1))
            assert_same(f"actions@{rep},{p}", cpu(acts[p]), r["actions"])
            assert_same(f"done@{rep},{p}", cpu(done[p]), r["done"])
            assert_same(f"outcome@{rep},{p}", cpu(outc[p]), r["outcome"])
            assert_same(f"reason@{rep},{p}", cpu(reas[p]), r["reason"])
            assert_same(f"ep_len@{rep},{p}", cpu(epl[p]), r["ep_len"])
        assert_same(f"last mask@{rep}", cpu(eng.mask), r["mask"])
        assert_same(f"last obs@{rep}", cpu(eng.obs), r["obs"])
        assert_same(f"states@{rep}", cpu(eng.export()), ref.export())
        t = cpu(ns)
        assert (t > 0).all()
    eng.close()


def test_plain_and_fused_engines_agree():
    n, seed = 512, 8
    a = E.Engine(n, seed, auto_reset=True, max_moves=1000)
    b = E.Engine(n, seed, auto_reset=True, max_moves=1000)
    for ply in range(30):
        a.legal_mask()
        a.sample()
        a.encode()
        a.step()
        E.stratego_run_plies(b.ctx, 1, mask=b.mask, actions=b.actions, obs=b.obs, done=b.done)
        assert_same(f"actions@{ply}", cpu(a.actions), cpu(b.actions))
        assert_same(f"obs@{ply}", cpu(a.obs), cpu(b.obs))
    assert_same("states", cpu(a.export()), cpu(b.export()))
    a.close()
    b.close()


def test_game_id_offset_shards_match_single_context():
    """Two contexts with game_id_base offsets reproduce one context's games."""
    n, seed = 1024, 9
    whole = E.Engine(n, seed, auto_reset=True, max_moves=1000)
    lo = E.Engine(n // 2, seed, auto_reset=True, max_moves=1000, game_id_base=0)
    hi = E.Engine(n // 2, seed, auto_reset=True, max_moves=1000, game_id_base=n // 2)
    for eng in (whole, lo, hi):
        E.stratego_run_plies(eng.ctx, 50, obs=eng.obs, use_graph=True)
    s = cpu(whole.export())
    assert_same("lo", cpu(lo.export()), s[: n // 2])
    assert_same("hi", cpu(hi.export()), s[n // 2:])
    for e in (whole, lo, hi):
        e.close()


# ---------------------------------------------------------------- play to the end
def test_4096_games_to_terminal_every_ply():
    """4096 games of random play without auto-reset until every game ends (or the
    1000-ply cap), one fused ply per launch.  Every ply, for every game: the
    mask, num_legal, action and step outputs, the record after the ply, and a
    digest of each observer's full observation (sum of the 48,800 bytes with
    SplitMix64 weights modulo 2^64, formed on the device and by the oracle
    library) equal the oracle's; the full observation bytes too at a few plies;
    then the outcome/reason and game-length histograms."""
    n, seed = 4096, 2
    eng = E.Engine(n, seed, k_battleless=100, max_moves=1000, auto_reset=False)
    ref = O.OracleEngine(n, seed, k_battleless=100, max_moves=1000, auto_reset=False)
    acts = torch.empty((1, n), dtype=torch.int16, device="cuda")
    done = torch.empty((1, n), dtype=torch.int8, device="cuda")
    outc = torch.empty((1, n), dtype=torch.int8, device="cuda")
    reas = torch.empty((1, n), dtype=torch.uint8, device="cuda")
    epl = torch.empty((1, n), dtype=torch.int16, device="cuda")
    ddig = DeviceDigest(torch, E.OBS_BYTES_PER_GAME // 2)
    obs_buf = np.empty((n, 2, 488, 10, 10), dtype=np.uint8)
    full_obs_at = {0, 1, 99, 399}
    ply = 0
    while True:
        E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, num_legal=eng.num_legal, actions=acts, obs=eng.obs,
                             done=done, outcome=outc, reason=reas, ep_len=epl)
        r = ref.ply(obs=True, mask=True, obs_out=obs_buf)
        assert_same(f"mask@{ply}", cpu(eng.mask), r["mask"])
        assert_same(f"num_legal@{ply}", cpu(eng.num_legal), r["num_legal"])
        assert_same(f"actions@{ply}", cpu(acts[0]), r["actions"])
        for name, t in (("done", done), ("outcome", outc), ("reason", reas), ("ep_len", epl)):
            assert_same(f"{name}@{ply}", cpu(t[0]), r[name])
        assert_same(f"obs digests@{ply}", ddig(eng.obs).reshape(n, 2),
                    O.digest_blocks(obs_buf, E.OBS_BYTES_PER_GAME // 2).reshape(n, 2))
        if ply in full_obs_at:
            assert_same(f"obs@{ply}", cpu(eng.obs), obs_buf)
        assert_same(f"records@{ply}", cpu(eng.export()), ref.export())
        ply += 1
        if cpu(done[0]).all():
            break
        assert ply <= 1000
    d_out, d_rsn, d_len = cpu(outc[0]), cpu(reas[0]), cpu(epl[0])
    recs = ref.export()
    hs = [header(recs[g]) for g in range(n)]
    want_pairs = np.zeros((3, 6), dtype=np.int64)
    got_pairs = np.zeros((3, 6), dtype=np.int64)
    for g in range(n):
        want_pairs[hs[g]["outcome"] + 1, hs[g]["reason"]] += 1
        got_pairs[int(d_out[g]) + 1, int(d_rsn[g])] += 1
    assert_same("outcome x reason histogram", got_pairs, want_pairs)
    assert_same("length histogram", np.bincount(d_len.astype(np.int64), minlength=1001),
                np.bincount(np.array([h["ply"] for h in hs]), minlength=1001))
    assert eng.error() == (0, -1)
    eng.close()


def test_device_digest_matches_the_oracle_digest():
    """The device-side digest forms the oracle library's sum: both on the same
    observation bytes, at two block sizes."""
    rng = np.random.default_rng(5)
    x = rng.integers(0, 256, size=(300, E.OBS_BYTES_PER_GAME // 2), dtype=np.uint8)
    x[rng.random(x.shape) < 0.9] = 0
    dev = torch.from_numpy(x).cuda()
    for block in (E.OBS_BYTES_PER_GAME // 2, E.OBS_BYTES_PER_GAME):
        assert_same(f"digest of {block}-byte blocks", DeviceDigest(torch, block, rows_per_chunk=37)(dev),
                    O.digest_blocks(x, block))


@pytest.mark.parametrize("n", [1, 7, 65, 1000, 5121, 20483])
def test_observation_free_plies_at_ragged_sizes(n):
    """The observation-free variant splits games statically and grows its
    tiles with N: odd sizes around the tile and wave counts, direct and from a
    graph, every ply's actions and the final states against the oracle."""
    seed = 31 + n
    eng = E.Engine(n, seed, k_battleless=20, max_moves=120, auto_reset=True)
    ref = O.OracleEngine(n, seed, k_battleless=20, max_moves=120, auto_reset=True)
    acts = torch.empty((8, n), dtype=torch.int16, device="cuda")
    for rnd in range(4):
        E.stratego_run_plies(eng.ctx, 8, actions=acts, use_graph=rnd % 2 == 1)
        for p in range(8):
            r = ref.ply(obs=False, mask=False)
            assert_same(f"actions@{rnd}.{p}", cpu(acts[p]), r["actions"])
    assert_same("states", cpu(eng.export()), ref.export())
    assert eng.error() == (0, -1)
    eng.close()


@pytest.mark.parametrize("sampler", [E.SAMPLER_UNIFORM, E.SAMPLER_MAGNET])
def test_observation_free_plies_beyond_64_games_per_wave(sampler):
    """Observation-free plies draw a wave's first 64 games ahead, one game per
    lane, and later games in the loop.  At 600,000 games a persistent launch
    gives every wave more than 64 games (256 CUs hold at most 8192 waves of
    this kernel), so both kinds of draw occur: every ply's actions and the
    final records equal the oracle's."""
    n, seed, plies = 600_000, 41, 3
    eng = E.Engine(n, seed, k_battleless=100, max_moves=1000, auto_reset=True, sampler=sampler)
    ref = O.OracleEngine(n, seed, k_battleless=100, max_moves=1000, auto_reset=True, sampler=sampler)
    acts = torch.empty((plies, n), dtype=torch.int16, device="cuda")
    E.stratego_run_plies(eng.ctx, plies, actions=acts)
    for p in range(plies):
        r = ref.ply(obs=False, mask=False)
        assert_same(f"actions@{p}", cpu(acts[p]), r["actions"])
    assert_same("states", cpu(eng.export()), ref.export())
    assert eng.error() == (0, -1)
    eng.close()


@pytest.mark.parametrize("n,with_mask", [(65, True), (5121, True), (1000, False)])
def test_observation_free_plies_write_every_output(n, with_mask):
    """Plies without observations, in the variant the rollouts use, with every
    per-game output asked for: the legal mask (or, without one, the legal
    count alone), action, done, outcome, reason and episode length equal the
    oracle's on every ply, one ply per call and from a graph of 32 plies.
    Short games (k = 20, 40 moves) make auto-resets and every end reason
    frequent."""
    seed = 71 + n
    eng = E.Engine(n, seed, k_battleless=20, max_moves=40, auto_reset=True)
    ref = O.OracleEngine(n, seed, k_battleless=20, max_moves=40, auto_reset=True)
    mask = eng.mask if with_mask else None
    keys = ("done", "outcome", "reason", "ep_len")
    ended = 0
    for ply in range(12):
        E.stratego_run_plies(eng.ctx, 1, mask=mask, num_legal=eng.num_legal, actions=eng.actions,
                             **{k: getattr(eng, k) for k in keys})
        r = ref.ply(obs=False, mask=with_mask)
        if with_mask:
            assert_same(f"mask@{ply}", cpu(mask), r["mask"])
        for k in ("num_legal", "actions") + keys:
            assert_same(f"{k}@{ply}", cpu(getattr(eng, k)), r[k])
    P = 32
    rows = {k: torch.full((P, n), -7, dtype=getattr(eng, k).dtype, device="cuda") for k in ("actions",) + keys}
    E.stratego_run_plies(eng.ctx, P, mask=mask, num_legal=eng.num_legal, use_graph=True, **rows)
    for p in range(P):
        r = ref.ply(obs=False, mask=with_mask)
        for k in ("actions",) + keys:
            assert_same(f"{k}@graph.{p}", cpu(rows[k][p]), r[k])
        ended += int((r["done"] != 0).sum())
    if with_mask:
        assert_same("mask@last", cpu(mask), r["mask"])
    assert_same("num_legal@last", cpu(eng.num_legal), r["num_legal"])
    assert_same("states", cpu(eng.export()), ref.export())
    assert ended > 0
    assert eng.error() == (0, -1)
    eng.close()


# ---------------------------------------------------------------- imported states
def random_position_records(count, seed=0):
    from test_oracle_pins import random_position
    rng = np.random.default_rng(seed)
    return np.stack([random_position(rng, int(rng.integers(1, 41)), int(rng.integers(1, 41)))
                     for _ in range(count)])


def test_masks_of_random_positions():
    recs = random_position_records(300)
    n = len(recs)
    eng = E.Engine(n, 1)
    eng.load(torch.from_numpy(recs).cuda())
    assert eng.error() == (0, -1)
    eng.legal_mask()
    ref = O.OracleEngine.from_records(recs, 1)
    m, nl = ref.mask()
    assert_same("mask", cpu(eng.mask), m)
    assert_same("num_legal", cpu(eng.num_legal), nl)
    assert_same("obs", cpu(eng.encode()), ref.encode())
    eng.close()


def scenario_records():
    from positions import T  # noqa: F401
    out = []
    out.append((make_record([dict(sq=sq(3, 1), owner=0, type="Captain"),
                             dict(sq=sq(4, 1), owner=1, type="Major", moved=1),
                             dict(sq=sq(0, 9), owner=0, type="Flag"),
                             dict(sq=sq(9, 9), owner=1, type="Flag")],
                            ply=2, moves=[(5, 15), (51, 41)]), 100 * 31 + 30))
    out.append((make_record([dict(sq=sq(3, 4), owner=0, type="Sergeant"),
                             dict(sq=sq(2, 5), owner=0, type="Captain"),
                             dict(sq=sq(4, 4), owner=1, type="General", revealed=1, moved=1),
                             dict(sq=sq(0, 9), owner=0, type="Flag"),
                             dict(sq=sq(9, 9), owner=1, type="Flag")],
                            ply=2, moves=[(3, 13), (54, 44)]), 100 * 25 + 35))
    out.append((make_record([dict(sq=sq(4, 4), owner=0, type="Marshal"),
                             dict(sq=sq(5, 4), owner=1, type="Captain"),
                             dict(sq=sq(6, 4), owner=1, type="Spy", revealed=1),
                             dict(sq=sq(4, 5), owner=1, type="Scout", revealed=1),
                             dict(sq=sq(0, 9), owner=0, type="Flag"),
                             dict(sq=sq(9, 9), owner=1, type="Flag")]), 100 * 44 + 54))
    for att, dfd, rdef in [("Sergeant", "Bomb", 0), ("Lieutenant", "Lieutenant", 1),
                           ("Captain", "Major", 1), ("Major", "Captain", 0), ("Spy", "Marshal", 0),
                           ("Miner", "Bomb", 1), ("Scout", "Flag", 0)]:
        out.append((make_record([dict(sq=sq(4, 4), owner=0, type=att),
                                 dict(sq=sq(5, 4), owner=1, type=dfd, revealed=rdef),
                                 dict(sq=sq(0, 0), owner=0, type="Flag"),
                                 dict(sq=sq(9, 9), owner=1, type="Flag") if dfd != "Flag" else
                                 dict(sq=sq(9, 9), owner=1, type="Bomb"),
                                 dict(sq=sq(9, 0), owner=1, type="Scout"),
                                 dict(sq=sq(0, 9), owner=0, type="Scout")], battleless=99),
                    100 * 44 + 54))
    return out


def test_hand_built_scenarios_step_like_the_oracle():
    sc = scenario_records()
    recs = np.stack([r for r, _ in sc])
    acts = np.array([a for _, a in sc], dtype=np.int16)
    n = len(sc)
    eng = E.Engine(n, 1)
    eng.load(torch.from_numpy(recs).cuda())
    eng.step(torch.from_numpy(acts).cuda())
    ref = O.OracleEngine.from_records(recs, 1)
    r = ref.step(acts)
    assert_same("states", cpu(eng.export()), ref.export())
    for k in ("done", "outcome", "reason", "ep_len"):
        assert_same(k, cpu(getattr(eng, k)), r[k])
    assert_same("obs", cpu(eng.encode()), ref.encode())
    assert eng.error() == (0, -1)
    eng.close()


def test_illegal_action_and_bad_record_are_latched():
    n = 16
    eng = E.Engine(n, 4)
    before = cpu(eng.export())
    acts = torch.full((n,), -1, dtype=torch.int16, device="cuda")
    acts[5] = 100 * 33 + 53          # not a legal move at ply 0
    acts[9] = 100 * 31 + 41
    eng.step(acts)
    rc, slot = eng.error()
    assert rc == E.E_ILLEGAL_ACTION and slot == 5
    after = cpu(eng.export())
    assert_same("untouched", after[5], before[5])
    assert eng.error() == (0, -1)
    bad = before[:2].copy()
    bad[1, 64 + 42] = 0               # a piece id on a lake square
    slots = torch.tensor([3, 7], dtype=torch.int32, device="cuda")
    eng.load(torch.from_numpy(bad).cuda(), slots)
    rc, slot = eng.error()
    assert rc == E.E_BAD_STATE and slot == 7
    now = cpu(eng.export())
    assert_same("slot 3 imported", now[3], before[0])
    assert_same("slot 7 kept", now[7], after[7])
    eng.close()


# ---------------------------------------------------------------- search-shaped load
def test_resample_and_rollout_262144_games():
    """1024 ply-100 states x 256 resamples, then 50 random plies: every record
    after resampling and after the rollout equals the oracle's."""
    seed, pool, per = 7, 4096, 256
    src_eng = O.OracleEngine(pool, seed, k_battleless=100, max_moves=1000)
    for _ in range(100):
        src_eng.ply(obs=False, mask=False)
    recs = src_eng.export()
    alive = [g for g in range(pool) if header(recs[g])["done"] == 0][:1024]
    assert len(alive) == 1024
    src = recs[alive]
    n = 1024 * per
    eng = E.Engine(n, seed, k_battleless=100, max_moves=1000)
    src_dev = torch.from_numpy(src).cuda()
    E.stratego_reset_resampled(eng.ctx, src_dev, per, 0)
    ref_src = O.OracleEngine.from_records(src, seed, max_moves=1000)
    ref = ref_src.resample(per, seed)
    assert_same("resampled", cpu(eng.export()), ref.export())
    E.stratego_run_plies(eng.ctx, 50, obs=None, use_graph=True)
    for _ in range(50):
        ref.ply(obs=False, mask=False)
    assert_same("after rollout", cpu(eng.export()), ref.export())
    eng.close()


def test_resample_edge_cases():
    """Sources of every kind (fresh setups: all hidden and unmoved; played
    records with moved, revealed and dead pieces and either side to move;
    sparse random positions), a per that is not a multiple of the resamples a
    wave takes, a nonzero game id base and spare slots: bit-exact with the
    oracle.  A malformed source is latched at its first slot and its slots
    are left alone."""
    seed, per, base = 11, 37, 1000
    fresh = O.OracleEngine(16, 5).export()
    ref = O.OracleEngine(64, 6, auto_reset=True)
    for _ in range(41):
        ref.ply(obs=False, mask=False)
    played = ref.export()
    sparse = random_position_records(48, seed=4)
    src = np.concatenate([fresh, played, sparse])
    nsrc = len(src)
    n = nsrc * per + 100
    eng = E.Engine(n, seed)
    before = cpu(eng.export())
    E.stratego_reset_resampled(eng.ctx, torch.from_numpy(src).cuda(), per, base)
    assert eng.error() == (0, -1)
    got = cpu(eng.export())
    want = O.OracleEngine.from_records(src, seed).resample(per, seed, base).export()
    assert_same("resampled", got[:nsrc * per], want)
    assert_same("spare slots", got[nsrc * per:], before[nsrc * per:])
    # a lake square holding a piece id: source 5 is refused
    bad = src.copy()
    bad[5, 64 + 42] = 0
    eng.load(torch.from_numpy(before).cuda())
    E.stratego_reset_resampled(eng.ctx, torch.from_numpy(bad).cuda(), per, base)
    assert eng.error() == (E.E_BAD_STATE, 5 * per)
    got = cpu(eng.export())
    rows = np.arange(nsrc * per)
    mine = (rows >= 5 * per) & (rows < 6 * per)
    assert_same("refused source's slots", got[:nsrc * per][mine], before[:nsrc * per][mine])
    assert_same("other sources", got[:nsrc * per][~mine], want[~mine])
    eng.close()


@pytest.mark.parametrize("per", [1, 64, 65, 129])
def test_resample_chunk_boundaries(per):
    """A wave draws up to 64 resamples of one source, one per lane: per
    around that chunk (a single resample, exactly one chunk, one chunk and a
    single resample, two chunks and one) gives the oracle's records."""
    seed, base = 19, 77
    ref = O.OracleEngine(40, 8, auto_reset=True)
    for _ in range(57):
        ref.ply(obs=False, mask=False)
    src = np.concatenate([O.OracleEngine(3, 9).export(), ref.export()])
    n = len(src) * per
    eng = E.Engine(n, seed)
    E.stratego_reset_resampled(eng.ctx, torch.from_numpy(src).cuda(), per, base)
    assert eng.error() == (0, -1)
    want = O.OracleEngine.from_records(src, seed).resample(per, seed, base).export()
    assert_same(f"resampled, per {per}", cpu(eng.export()), want)
    eng.close()


def test_resample_then_magnet_rollouts():
    """The search-shaped load with magnet-policy rollouts (section 2.4): 64
    mid-game states x 16 resamples, 50 plies in a captured graph, every
    record after the rollout and the last ply's outcomes equal the oracle's."""
    seed, per, plies = 13, 16, 50
    src_eng = O.OracleEngine(256, seed, k_battleless=100, max_moves=1000)
    for _ in range(60):
        src_eng.ply(obs=False, mask=False)
    recs = src_eng.export()
    alive = [g for g in range(256) if header(recs[g])["done"] == 0][:64]
    src = recs[alive]
    n = len(src) * per
    eng = E.Engine(n, seed, k_battleless=100, max_moves=1000, sampler=E.SAMPLER_MAGNET)
    E.stratego_reset_resampled(eng.ctx, torch.from_numpy(src).cuda(), per, 0)
    done = torch.empty((plies, n), dtype=torch.int8, device="cuda")
    outc = torch.empty((plies, n), dtype=torch.int8, device="cuda")
    E.stratego_run_plies(eng.ctx, plies, done=done, outcome=outc, use_graph=True)
    ref = O.OracleEngine.from_records(src, seed, max_moves=1000, sampler=O.SAMPLER_MAGNET).resample(per, seed)
    for _ in range(plies - 1):
        ref.ply(obs=False, mask=False)
    r = ref.ply(obs=False, mask=False)
    assert_same("states after magnet rollouts", cpu(eng.export()), ref.export())
    assert_same("done", cpu(done[-1]), r["done"])
    assert_same("outcome", cpu(outc[-1]), r["outcome"])
    assert eng.error() == (0, -1)
    eng.close()


# ---------------------------------------------------------------- serving
def serving_inputs(total, seed=2):
    """Start states drawn from games of random play without auto-reset (the
    4096-game workload), taken at different plies."""
    ref = O.OracleEngine(2048, seed, k_battleless=100, max_moves=1000)
    pool = []
    for ply in range(121):
        ref.ply(obs=False, mask=False)
        if ply % 40 == 0:
            pool.append(ref.export())
    pool = np.concatenate(pool)
    rng = np.random.default_rng(seed)
    return pool[rng.choice(len(pool), size=total, replace=False)]


def test_serving_results_same_alone_and_in_the_mix():
    """Continuous batching over a 4096-slot pool with a small memory budget:
    every request's final states (and step requests' observations) equal the
    same request served alone and the oracle's."""
    rng = np.random.default_rng(5)
    sizes = [1, 7, 64, 300, 1000, 5, 129, 700, 33, 2, 411, 90]
    reqs, first, t = [], 0, 0.0
    for r, b in enumerate(sizes):
        kind = E.REQ_STEP if r % 2 == 0 else E.REQ_ROLLOUT
        plies = 1 if kind == E.REQ_STEP else int(rng.integers(1, 41))
        t += float(rng.exponential(0.002))
        reqs.append((kind, plies, b, first, t))
        first += b
    total = first
    recs = serving_inputs(total)
    seed = 2
    eng = E.Engine(4096, seed, k_battleless=100, max_moves=1000, auto_reset=False)
    inp = torch.from_numpy(recs).cuda()
    out_mix = torch.zeros_like(inp)
    obs_mix = torch.zeros((total, 2, 488, 10, 10), dtype=torch.uint8, device="cuda")
    budget = 1500 * 1536 + 1000 * 97600          # forces requests to queue
    res, stats = E.stratego_serve(eng.ctx, reqs, inp, out_mix, obs_mix, mem_budget_bytes=budget,
                                  realtime=True)
    assert eng.error() == (0, -1)
    assert stats["game_steps"] == sum(b * p for _, p, b, _, _ in reqs)
    assert stats["peak_reserved_bytes"] <= budget
    assert 0 < stats["gpu_busy_s"] <= stats["gpu_span_s"] * 1.001 and stats["gpu_span_s"] <= stats["wall_s"]
    for (a, d), q in zip(res, reqs):
        assert q[4] <= a + 1e-3 and a <= d
    out_mix_h, obs_mix_h = cpu(out_mix), cpu(obs_mix)
    for r, q in enumerate(reqs):
        kind, plies, b, f, _ = q
        out_one = torch.zeros_like(inp)
        obs_one = torch.zeros_like(obs_mix)
        E.stratego_serve(eng.ctx, [(kind, plies, b, f, 0.0)], inp, out_one, obs_one, realtime=False)
        assert_same(f"request {r} states alone vs mix", cpu(out_one)[f:f + b], out_mix_h[f:f + b])
        if kind == E.REQ_STEP:
            assert_same(f"request {r} obs alone vs mix", cpu(obs_one)[f:f + b], obs_mix_h[f:f + b])
        ref = O.OracleEngine.from_records(recs[f:f + b], seed, k_battleless=100, max_moves=1000)
        for p in range(plies):
            rr = ref.ply(obs=(kind == E.REQ_STEP), mask=False)
        assert_same(f"request {r} vs oracle", out_mix_h[f:f + b], ref.export())
        if kind == E.REQ_STEP:
            assert_same(f"request {r} obs vs oracle", obs_mix_h[f:f + b], rr["obs"])
    eng.close()


def test_serving_observations_by_slot():
    """obs_by_slot = 1 (as the serving benchmark runs): a step request's
    observations land at the pool slots its games occupy.  With a pool larger
    than all requests together and every request there at the start, no slot
    is reused, so the rows written are exactly the oracle's observations of the
    step requests' input states (compared as a set of rows: which slot a game
    takes is the loop's own choice), and the other rows keep their fill."""
    seed, N, fill = 2, 256, 0x5A
    reqs = [(E.REQ_STEP, 1, 20, 0, 0.0), (E.REQ_ROLLOUT, 3, 50, 20, 0.0), (E.REQ_STEP, 1, 13, 70, 0.0)]
    total = 83
    recs = serving_inputs(total)
    eng = E.Engine(N, seed, k_battleless=100, max_moves=1000, auto_reset=False)
    inp = torch.from_numpy(recs).cuda()
    out = torch.zeros_like(inp)
    pool = torch.full((N, 2, 488, 10, 10), fill, dtype=torch.uint8, device="cuda")
    E.stratego_serve(eng.ctx, reqs, inp, out, pool, obs_by_slot=True, realtime=False)
    assert eng.error() == (0, -1)
    got = cpu(pool).reshape(N, -1)
    written = got[(got != fill).any(axis=1)]
    want = np.concatenate([
        O.OracleEngine.from_records(recs[f:f + b], seed, k_battleless=100, max_moves=1000).ply(obs=True, mask=False)["obs"]
        for kind, _, b, f, _ in reqs if kind == E.REQ_STEP]).reshape(33, -1)
    assert len(written) == len(want) == 33
    key = lambda a: sorted(r.tobytes() for r in a)
    assert key(written) == key(want), "the observation rows written differ from the oracle's"
    out_h = cpu(out)
    for kind, plies, b, f, _ in reqs:
        ref = O.OracleEngine.from_records(recs[f:f + b], seed, k_battleless=100, max_moves=1000)
        for _ in range(plies):
            ref.ply(obs=False, mask=False)
        assert_same(f"request at row {f} vs oracle", out_h[f:f + b], ref.export())
    eng.close()


def test_serving_backfill_admits_smaller_requests_first():
    """Admission order with and without backfilling, on a 100-slot pool: a
    50-game request that cannot fit beside a running 90-game one holds back a
    later 5-game request in strict arrival order, and lets it go ahead with
    backfilling.  Every request's final states are the same either way."""
    recs = serving_inputs(145)
    inp = torch.from_numpy(recs).cuda()
    reqs = [(E.REQ_ROLLOUT, 20, 90, 0, 0.0),     # fills 90 of the 100 slots for 20 plies
            (E.REQ_ROLLOUT, 1, 50, 90, 0.0),     # does not fit until it leaves
            (E.REQ_STEP, 1, 5, 140, 0.0)]        # fits beside it
    outs, admits = {}, {}
    for name, wait in (("strict", -1.0), ("backfill", 10.0)):
        eng = E.Engine(100, 3, k_battleless=100, max_moves=1000, auto_reset=False)
        out = torch.zeros_like(inp)
        obs = torch.zeros((145, 2, 488, 10, 10), dtype=torch.uint8, device="cuda")
        res, stats = E.stratego_serve(eng.ctx, reqs, inp, out, obs, realtime=False, backfill_wait_s=wait)
        assert eng.error() == (0, -1)
        assert stats["peak_active_games"] <= 100
        admits[name] = [a for a, _ in res]
        outs[name] = cpu(out)
        eng.close()
    s_adm, b_adm = admits["strict"], admits["backfill"]
    assert s_adm[0] <= s_adm[1] <= s_adm[2], s_adm       # arrival order
    assert b_adm[2] < b_adm[1], b_adm                    # the 5 games went ahead
    assert_same("final states, strict vs backfill", outs["strict"], outs["backfill"])


# ---------------------------------------------------------------- full size
def test_65536_games_whole_population_graph_plies():
    """The benchmark's configuration (65,536 games, auto-reset, autotuned
    tiling, 64-ply hipGraph launches) against the oracle playing all 65,536
    games: over 192 plies every game's action, done flag and outcome every
    ply, every record after each graph launch, and at the last ply every
    game's mask and both observations, byte for byte."""
    n, seed, P, launches = 65536, 1, 64, 3
    eng = E.Engine(n, seed, k_battleless=100, max_moves=1000, auto_reset=True)
    E.stratego_autotune(eng.ctx, eng.obs, eng.mask, plies=2)
    G, S = E.stratego_get_tiling(eng.ctx)
    print(f"tiling G={G} layout={S}", flush=True)
    acts = torch.empty((P, n), dtype=torch.int16, device="cuda")
    done = torch.empty((P, n), dtype=torch.int8, device="cuda")
    outc = torch.empty((P, n), dtype=torch.int8, device="cuda")
    ref = O.OracleEngine(n, seed, k_battleless=100, max_moves=1000, auto_reset=True)
    chunk = 4096
    for launch in range(launches):
        E.stratego_run_plies(eng.ctx, P, mask=eng.mask, actions=acts, obs=eng.obs, done=done, outcome=outc,
                             use_graph=True)
        a_h, d_h, o_h = cpu(acts), cpu(done), cpu(outc)
        for p in range(P):
            ply = launch * P + p
            last = launch == launches - 1 and p == P - 1
            if last:   # the last ply's observations and mask are of its pre-move states
                for g0 in range(0, n, chunk):
                    idx = np.arange(g0, g0 + chunk, dtype=np.int32)
                    assert_same(f"obs@{ply} games {g0}..", cpu(eng.obs[g0:g0 + chunk]), ref.encode(idx))
            r = ref.ply(obs=False, mask=last)
            assert_same(f"actions@{ply}", a_h[p], r["actions"])
            assert_same(f"done@{ply}", d_h[p], r["done"])
            assert_same(f"outcome@{ply}", o_h[p], r["outcome"])
            if last:
                assert_same(f"mask@{ply}", cpu(eng.mask), r["mask"])
        assert_same(f"records after ply {launch * P + P - 1}", cpu(eng.export()), ref.export())
    assert eng.error() == (0, -1)
    eng.close()


def test_65536_games_after_1024_plies_sampled():
    """The desynchronised regime the benchmark times: 65,536 games, auto-reset,
    autotuned tiling, 1,088 plies from 64-ply graphs; 2,048 games spread over
    the slots, each checked against the oracle playing only those game ids:
    the last 64 plies' actions and done flags, the final records, and the last
    ply's mask and both observations."""
    n, seed, P = 65536, 3, 64
    eng = E.Engine(n, seed, k_battleless=100, max_moves=1000, auto_reset=True)
    E.stratego_autotune(eng.ctx, eng.obs, eng.mask, plies=2)
    acts = torch.empty((P, n), dtype=torch.int16, device="cuda")
    done = torch.empty((P, n), dtype=torch.int8, device="cuda")
    launches = 17
    for _ in range(launches):
        E.stratego_run_plies(eng.ctx, P, mask=eng.mask, actions=acts, obs=eng.obs, done=done, use_graph=True)
    rng = np.random.default_rng(7)
    ids = np.sort(rng.choice(n, size=2048, replace=False)).astype(np.int64)
    idx = torch.from_numpy(ids).cuda()
    ref = O.OracleEngine(len(ids), seed, k_battleless=100, max_moves=1000, auto_reset=True,
                         game_ids=ids.astype(np.uint32))
    total = launches * P
    for p in range(total):
        last = p == total - 1
        r = ref.ply(obs=last, mask=last)
        if p >= total - P:
            assert_same(f"actions@{p}", cpu(acts[p - total + P].index_select(0, idx)), r["actions"])
            assert_same(f"done@{p}", cpu(done[p - total + P].index_select(0, idx)), r["done"])
    assert_same("last mask", cpu(eng.mask.index_select(0, idx)), r["mask"])
    assert_same("last obs", cpu(eng.obs.index_select(0, idx)), r["obs"])
    recs = cpu(eng.export().index_select(0, idx))
    assert_same("records", recs, ref.export())
    hs = [header(recs[g]) for g in range(len(ids))]
    # desynchronised: every game has restarted (no game lasts more than 1000
    # plies) and the games stand at many different plies of their episodes
    assert min(h["episode"] for h in hs) >= 1
    assert len({h["ply"] for h in hs}) > 300
    assert eng.error() == (0, -1)
    eng.close()


@pytest.mark.parametrize("G,L", [(1, 1), (4, 5), (2, 7)])
def test_acting_player_observations(G, L):
    """acting_obs_only: the fused ply, the plain encoder and the rollout
    buffer's query write only the acting player's information state (App. B.1
    ComputeInfostateTensor), bit-exact with the oracle's."""
    n, seed = 700, 13
    kw = dict(k_battleless=100, max_moves=1000, auto_reset=True)
    eng = E.Engine(n, seed, acting_obs=True, games_per_wg=G, lds_layout=L, history_len=4, **kw)
    ref = O.OracleEngine(n, seed, acting_obs=True, **kw)
    assert tuple(eng.obs.shape) == (n, 1, 488, 10, 10)
    for ply in range(30):
        E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, actions=eng.actions, obs=eng.obs)
        r = ref.ply(obs=True)
        assert_same(f"actions@{ply}", cpu(eng.actions), r["actions"])
        assert_same(f"obs@{ply}", cpu(eng.obs), r["obs"])
    last = cpu(eng.obs)
    assert_same("plain encoder", cpu(eng.encode()), ref.encode())
    lo, T = eng.window()
    assert_same("history obs at T-1", cpu(eng.obs_at(T - 1)), last)
    eng.close()
