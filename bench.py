"""Benchmark of the batched Stratego engine on one MI355X.

Metric: game steps per second at 65,536 games, where one game step is a legal
mask of the player to move + a uniform Philox sample + the step (battle,
terminal and draw checks, auto-reset) + the uint8 observation encoding
[2, 488, 10, 10] of both players.  The timed engine is the fused persistent
kernel, one launch per ply, replayed from hipGraphs of up to 64 plies; exactly
--steps plies are timed after exactly --warmup plies.  Inputs are
synthetic: uniform random setups from the seed and uniform random legal play.

Prints one JSON line.  Also reports per-ply p50/p99 latency (device
timestamps), the HBM roofline fraction of the fused ply kernel, the plain
per-call engine at the same size, serving under load, the rollout buffer
(recording plies and queries at past steps), the competitive-play rules, the
policy kernels, the acting-player-only variant, the search-shaped load
(resampling and rollouts at 262,144 games), the autotuner table and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GAMES = 65536
GRAPH_PLIES = 64
K_BATTLELESS = 100
MAX_MOVES = 1000
SEED = 1
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of one game step of the fused ply: obs 97600 written,
# mask 1256 written, num_legal 2, action 2, done/outcome/reason/ep_len 5,
# state record 1536 read + 1536 written
BYTES_PER_GAME_STEP = 97600 + 1256 + 2 + 2 + 5 + 2 * 1536
EXTRA_LEGS = ("rollout_buffer", "rules", "policies", "acting", "search", "steady", "small")


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def graph_split(steps):
    """The timed plies run from `full` graphs of P plies and, for the
    remainder, one graph of R plies: P * full + R == steps exactly."""
    P = min(GRAPH_PLIES, steps)
    full, R = divmod(steps, P)
    return P, full, R


def traffic_from_profile():
    """HBM bytes per launch measured by rocprofv3 counters for the current
    kernel source, or None when no such measurement exists."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "fused_ply_65536_traffic.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ("device.h", "engine.hip"):
        h.update(open(os.path.join(ROOT, "paper_2511_07312_amd", "csrc", f), "rb").read())
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != h.hexdigest():
        return None
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(seconds=12.0):
    """The CPU oracle on the host cores, same workload definition (fused ply
    with both observations, auto-reset) on a bounded sample of games."""
    import numpy as np
    import oracle
    n = 4096
    ref = oracle.OracleEngine(n, SEED, K_BATTLELESS, MAX_MOVES, auto_reset=True)
    for _ in range(64):                      # advance past the opening (no encode)
        ref.ply(obs=False, mask=False)
    plies = 0
    t0 = time.perf_counter()
    while True:
        ref.ply(obs=True)
        plies += 1
        el = time.perf_counter() - t0
        if el >= seconds or plies >= 20000:
            break
    cores = oracle.num_threads()
    return dict(value=n * plies / el, unit="game steps/s", cores=cores, per_core=n * plies / el / cores,
                kind="oracle",
                sample=f"games 0..{n - 1} of the same seed, {plies} fused plies each (mask, sample, "
                       f"encode both players, step, auto-reset) after 64 unencoded plies; "
                       f"{el:.1f} s wall")


def serving_bench(E, torch, n_requests=2000, seed=4, backfill_wait_s=0.005):
    """Continuous-batching serving: Poisson arrivals, half step requests (one
    ply with both observations) and half k-ply rollouts (k uniform in 1..128),
    batch sizes floor(exp(U(0, ln 16384))), start states drawn from games of
    random play without auto-reset.  Admission backfills: a request that does
    not fit lets later ones go ahead for up to backfill_wait_s (< 0: strict
    arrival order).  Measures the saturated rate, then p50/p99 latency and
    throughput at 0.3, 0.6 and 0.9 of it."""
    import math
    import numpy as np
    rng = np.random.default_rng(seed)
    # start-state pool from 4096 games of random play (no auto-reset)
    src = E.Engine(4096, 2, K_BATTLELESS, MAX_MOVES, auto_reset=False)
    pool = []
    for _ in range(5):
        E.stratego_run_plies(src.ctx, 30, obs=None, use_graph=True)
        pool.append(src.export())
    pool = torch.cat(pool)
    src.close()
    kinds = rng.integers(0, 2, size=n_requests)
    sizes = np.floor(np.exp(rng.uniform(0, math.log(16384), size=n_requests))).astype(int)
    plies = np.where(kinds == 0, 1, rng.integers(1, 129, size=n_requests))
    firsts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    total = int(sizes.sum())
    rows = torch.from_numpy(rng.integers(0, pool.shape[0], size=total)).cuda()
    inp = pool[rows].contiguous()
    out = torch.empty_like(inp)
    slots = 65536
    eng = E.Engine(slots, 2, K_BATTLELESS, MAX_MOVES, auto_reset=False)
    obs_pool = torch.empty((slots, 2, 488, 10, 10), dtype=torch.uint8, device="cuda")
    gaps = rng.exponential(1.0, size=n_requests)

    def run(rate):
        arr = np.zeros(n_requests) if rate is None else np.cumsum(gaps) / rate
        reqs = [(int(kinds[r]), int(plies[r]), int(sizes[r]), int(firsts[r]), float(arr[r]))
                for r in range(n_requests)]
        res, st = E.stratego_serve(eng.ctx, reqs, inp, out, obs_pool, obs_by_slot=True,
                                   mem_budget_bytes=0, realtime=rate is not None,
                                   backfill_wait_s=backfill_wait_s)
        lat = {0: [], 1: []}
        for r, (a, d) in enumerate(res):
            lat[int(kinds[r])].append((d - arr[r]) * 1e3)
        return st, lat

    st, _ = run(None)
    sat = st["game_steps"] / st["wall_s"]
    sat_idle = 1.0 - st["gpu_busy_s"] / st["gpu_span_s"] if st["gpu_span_s"] > 0 else None
    mean_work = float((sizes * plies).mean())
    out_rates = []
    for f in (0.3, 0.6, 0.9):
        rate = f * sat / mean_work            # requests per second
        st, lat = run(rate)
        out_rates.append(dict(
            load=f, requests_per_s=rate, throughput=st["game_steps"] / st["wall_s"],
            step_p50_ms=percentile(lat[0], 0.5), step_p99_ms=percentile(lat[0], 0.99),
            rollout_p50_ms=percentile(lat[1], 0.5), rollout_p99_ms=percentile(lat[1], 0.99),
            gpu_idle_fraction=1.0 - st["gpu_busy_s"] / st["gpu_span_s"] if st["gpu_span_s"] > 0 else None,
            iterations=st["iterations"], peak_active_games=st["peak_active_games"]))
        print(f"[bench] serving at {f:.1f}x: {out_rates[-1]}", file=sys.stderr, flush=True)
    assert eng.error() == (0, -1)
    eng.close()
    return dict(unit="game steps/s", saturated=sat, saturated_gpu_idle_fraction=sat_idle,
                requests=n_requests, games=total, backfill_wait_s=backfill_wait_s,
                pool_slots=slots, rates=out_rates)


def rollout_buffer_bench(E, torch, n=GAMES, H=64, warm=256):
    """Rollout-buffer mode (App. B.1): plies without observations record each
    game's state in a ring of H steps; masks and information states of past
    steps are re-materialised on demand.  Times recording plies (against the
    same plies without a ring) and the queries at a past step, all N games."""
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn, reps):
        fn()
        ev[0].record(stream)
        for _ in range(reps):
            fn()
        ev[1].record(stream)
        ev[1].synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    res = {}
    for hl in (0, H):
        eng = E.Engine(n, SEED, K_BATTLELESS, MAX_MOVES, auto_reset=True, history_len=hl)
        acts = torch.empty((GRAPH_PLIES, n), dtype=torch.int16, device="cuda")
        done = torch.empty((GRAPH_PLIES, n), dtype=torch.int8, device="cuda")
        outc = torch.empty((GRAPH_PLIES, n), dtype=torch.int8, device="cuda")

        def plies():
            E.stratego_run_plies(eng.ctx, GRAPH_PLIES, actions=acts, done=done, outcome=outc,
                                 use_graph=True)
        for _ in range(warm // GRAPH_PLIES):
            plies()
        res[hl] = timed(plies, 4) / GRAPH_PLIES
        if hl:
            lo, T = eng.window()
            t = T - H // 2
            obs = torch.empty((n, 2, 488, 10, 10), dtype=torch.uint8, device="cuda")
            mask = torch.empty((n, 157), dtype=torch.int64, device="cuda")
            nl = torch.empty(n, dtype=torch.int16, device="cuda")
            info = {k: torch.empty(n * per, dtype=dt, device="cuda") for k, (dt, per) in E.HISTORY_INFO.items()
                    if per == 1}
            obs_ms = timed(lambda: E.stratego_history_encode_obs(eng.ctx, t, obs, None, n), 8)
            mask_ms = timed(lambda: E.stratego_history_legal_mask(eng.ctx, t, mask, nl, None, n), 8)
            info_ms = timed(lambda: E.stratego_history_info(eng.ctx, t, None, n, **info), 8)
            assert eng.error() == (0, -1)
            del obs, mask, nl, info
        eng.close()
        torch.cuda.empty_cache()
    q_bytes = (97600 + 1536) * n
    out = dict(
        games=n, history_len=H,
        ring_bytes=H * n * 1544,
        stored_equivalent_bytes=H * n * (97600 + 1256),
        record_ply_ms=res[H], plain_ply_ms=res[0],
        recording_overhead=res[H] / res[0] - 1.0,
        record_game_steps_per_s=n / (res[H] / 1e3),
        obs_query_ms=obs_ms, obs_query_games_per_s=n / (obs_ms / 1e3),
        obs_query_roofline=dict(bound="hbm", achieved=q_bytes / (obs_ms / 1e3) / 1e9, peak=HBM_PEAK_GBS,
                                unit="GB/s", frac=q_bytes / (obs_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                                bytes_per_game=97600 + 1536, kernel="k_hist<1> (information states at t)"),
        mask_query_ms=mask_ms, info_query_ms=info_ms,
        query_step="t = current - H/2 (a ring row, not the live states)",
    )
    print(f"[bench] rollout buffer: {out}", file=sys.stderr, flush=True)
    return out


def two_square_bench(E, torch, n=GAMES, warm=256, timed=128):
    """The fused ply with both competitive-play rules on (App. A: two-square
    and continuous chasing): same workload as the headline run, rules
    enforced in masks and terminal tests; also the share of games each rule
    restricts at the end."""
    eng = E.Engine(n, SEED, K_BATTLELESS, MAX_MOVES, auto_reset=True, two_square=True, chasing=True)
    obs = eng.obs

    def plies():
        E.stratego_run_plies(eng.ctx, GRAPH_PLIES, obs=obs, use_graph=True)
    for _ in range(warm // GRAPH_PLIES):
        plies()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(timed // GRAPH_PLIES):
        plies()
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / timed
    ts = torch.empty(n, dtype=torch.uint8, device="cuda")
    ch = torch.empty(n, dtype=torch.uint8, device="cuda")
    E.stratego_history_info(eng.ctx, eng.window()[1], None, n, two_square_applies=ts, chase_applies=ch)
    assert eng.error() == (0, -1)
    eng.close()
    out = dict(ms_per_ply=ms, game_steps_per_s=n / (ms / 1e3), two_square_share=float(ts.float().mean()),
               chase_share=float(ch.float().mean()),
               workload=f"{n} games, fused ply with observations, two-square and chasing rules on")
    print(f"[bench] competitive rules: {out}", file=sys.stderr, flush=True)
    return out


def policy_bench(E, torch, n=GAMES, warm=256, timed=128):
    """Sections 2.4-2.5 / App. D.7 at the headline size: the fused ply with the
    magnet sampler, and the legal-list policy kernels (magnet probabilities,
    the search policy with the paper's alpha = 0.002, beta = 0.02, and the
    sampler over it) on 65,536 mid-game positions."""
    eng = E.Engine(n, SEED, K_BATTLELESS, MAX_MOVES, auto_reset=True, sampler=E.SAMPLER_MAGNET)
    obs = eng.obs
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed_ms(fn, reps):
        fn()
        ev[0].record(stream)
        for _ in range(reps):
            fn()
        ev[1].record(stream)
        ev[1].synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    def plies():
        E.stratego_run_plies(eng.ctx, GRAPH_PLIES, obs=obs, use_graph=True)
    for _ in range(warm // GRAPH_PLIES):
        plies()
    ply_ms = timed_ms(plies, timed // GRAPH_PLIES) / GRAPH_PLIES
    del obs
    eng._obs = None
    torch.cuda.empty_cache()
    acts = torch.empty((n, E.MAX_LEGAL), dtype=torch.int16, device="cuda")
    nl = torch.empty(n, dtype=torch.int16, device="cuda")
    probs = torch.empty((n, E.MAX_LEGAL), dtype=torch.float32, device="cuda")
    q = torch.rand((n, E.MAX_LEGAL), dtype=torch.float32, device="cuda") * 2 - 1
    logpi = torch.full((n, E.MAX_LEGAL), -3.0, dtype=torch.float32, device="cuda")
    picks = torch.empty(n, dtype=torch.int16, device="cuda")
    list_ms = timed_ms(lambda: E.stratego_legal_list(eng.ctx, acts, nl), 8)
    magnet_ms = timed_ms(lambda: E.stratego_magnet_policy(eng.ctx, probs), 8)
    search_ms = timed_ms(lambda: E.stratego_search_policy(eng.ctx, q, logpi, 0.002, 0.02, probs), 8)
    sample_ms = timed_ms(lambda: E.stratego_sample_policy(eng.ctx, probs, picks), 8)
    assert eng.error() == (0, -1)
    eng.close()
    out = dict(magnet_ply_ms=ply_ms, magnet_game_steps_per_s=n / (ply_ms / 1e3),
               legal_list_ms=list_ms, magnet_policy_ms=magnet_ms, search_policy_ms=search_ms,
               sample_policy_ms=sample_ms, positions=n,
               workload=f"{n} games, fused ply with observations and the magnet sampler; "
                        "policy kernels on the resulting positions")
    print(f"[bench] policies: {out}", file=sys.stderr, flush=True)
    return out


def acting_player_bench(E, torch, n=GAMES, warm=256, timed=320):
    """Secondary metric: the same fused ply writing only the acting player's
    information state ([N, 1, 488, 10, 10], App. B.1 ComputeInfostateTensor)."""
    eng = E.Engine(n, SEED, K_BATTLELESS, MAX_MOVES, auto_reset=True, acting_obs=True)
    obs = eng.obs
    ply_ns = torch.empty(GRAPH_PLIES, dtype=torch.int64, device="cuda")

    def plies(timed_run):
        E.stratego_run_plies(eng.ctx, GRAPH_PLIES, mask=eng.mask, obs=obs, use_graph=True,
                             ply_ns=ply_ns if timed_run else None)
    for _ in range(warm // GRAPH_PLIES):
        plies(False)
    tune = E.stratego_autotune(eng.ctx, obs, eng.mask, plies=4)
    G, S = E.stratego_get_tiling(eng.ctx)
    plies(True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lat = []
    e0.record(stream)
    for _ in range(timed // GRAPH_PLIES):
        plies(True)
        lat += [x / 1e6 for x in ply_ns.cpu().tolist()]
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / timed
    assert eng.error() == (0, -1)
    eng.close()
    bytes_per_step = 48800 + 1256 + 2 + 5 + 2 * 1536
    achieved = bytes_per_step * n / (ms / 1e3) / 1e9
    out = dict(value=n / (ms / 1e3), unit="game steps/s", ms_per_step=ms, p50_ms=percentile(lat, 0.5),
               p99_ms=percentile(lat, 0.99), bytes_per_game_step=bytes_per_step,
               achieved_GBs=achieved, frac=achieved / HBM_PEAK_GBS, games_per_wg=G, lds_layout=S,
               autotune=[dict(games_per_wg=g, lds_layout=s_, us_per_ply=u) for g, s_, u in tune],
               workload=f"{n} games, fused ply, acting player's observations only")
    print(f"[bench] acting player only: {out}", file=sys.stderr, flush=True)
    return out


def search_bench(E, torch, n_src=1024, per=256, plies=50, reps=4):
    """The search-shaped load (section 2.5 / App. B): 1024 mid-game states
    from random play to ply 100, 256 resamples of the opponent's hidden
    pieces each (262,144 games materialised on the device), then 50 random
    plies of every resampled game with their per-ply outcomes."""
    pool = 4096
    src_eng = E.Engine(pool, SEED, K_BATTLELESS, MAX_MOVES, auto_reset=False)
    E.stratego_run_plies(src_eng.ctx, 100, use_graph=True)
    recs = src_eng.export()
    live = torch.nonzero(recs[:, 17] == 0).flatten()[:n_src]
    assert live.numel() == n_src, live.numel()
    src = recs[live].contiguous()
    src_eng.close()
    n = n_src * per
    eng = E.Engine(n, SEED, K_BATTLELESS, MAX_MOVES, auto_reset=False)
    done = torch.empty((plies, n), dtype=torch.int8, device="cuda")
    outc = torch.empty((plies, n), dtype=torch.int8, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def load():
        E.stratego_reset_resampled(eng.ctx, src, per, 0)
        E.stratego_run_plies(eng.ctx, plies, done=done, outcome=outc, use_graph=True)
    load()                                   # captures the rollout graph
    res_ms, roll_ms = [], []
    for _ in range(reps):
        ev[0].record(stream)
        E.stratego_reset_resampled(eng.ctx, src, per, 0)
        ev[1].record(stream)
        E.stratego_run_plies(eng.ctx, plies, done=done, outcome=outc, use_graph=True)
        ev[2].record(stream)
        ev[2].synchronize()
        res_ms.append(ev[0].elapsed_time(ev[1]))
        roll_ms.append(ev[1].elapsed_time(ev[2]))
    ended = float((done[-1] != 0).float().mean())
    assert eng.error() == (0, -1)
    eng.close()
    # the same load with magnet-policy rollouts (section 2.4), the paper's
    # rollout policy before a network is trained
    eng = E.Engine(n, SEED, K_BATTLELESS, MAX_MOVES, auto_reset=False, sampler=E.SAMPLER_MAGNET)
    load()
    magnet_ms = []
    for _ in range(reps):
        E.stratego_reset_resampled(eng.ctx, src, per, 0)
        ev[1].record(stream)
        E.stratego_run_plies(eng.ctx, plies, done=done, outcome=outc, use_graph=True)
        ev[2].record(stream)
        ev[2].synchronize()
        magnet_ms.append(ev[1].elapsed_time(ev[2]))
    assert eng.error() == (0, -1)
    eng.close()
    r, w = min(res_ms), min(roll_ms)
    # resample: each new record (1536 B) written, its source read once per
    # game from cache; rollout ply: record read + written, done + outcome
    res_bytes = n * 1536 + n_src * 1536
    out = dict(games=n, resample_ms=r, resample_GBs=res_bytes / (r / 1e3) / 1e9,
               rollout_ms=w, rollout_ms_per_ply=w / plies,
               rollout_game_steps_per_s=n * plies / (w / 1e3), total_ms=r + w,
               resampled_states_per_s=n / (r / 1e3), ended_within_50_plies=ended,
               magnet_rollout_ms=min(magnet_ms),
               magnet_rollout_game_steps_per_s=n * plies / (min(magnet_ms) / 1e3),
               workload=f"{n_src} ply-100 states x {per} resamples, {plies} random plies each "
                        "(no observations), best of {reps} runs".replace("{reps}", str(reps)))
    print(f"[bench] search-shaped load: {out}", file=sys.stderr, flush=True)
    return out


def steady_state_bench(E, torch, G, S, n=GAMES, seeds=(1, 2, 3), warm=1024, timed=640):
    """The headline workload at its steady state, per seed (the tuned tiling):
    1024 plies first, so that the games' episodes have desynchronised (random
    games last about 490 plies on average and at most 1000, and every game
    restarts on its own), then 640 timed plies from graphs of 64."""
    out = {}
    stream = torch.cuda.current_stream()
    for seed in seeds:
        eng = E.Engine(n, seed, K_BATTLELESS, MAX_MOVES, auto_reset=True)
        E.stratego_set_tiling(eng.ctx, G, S)
        obs = eng.obs

        def plies():
            E.stratego_run_plies(eng.ctx, GRAPH_PLIES, mask=eng.mask, obs=obs, use_graph=True)
        for _ in range(warm // GRAPH_PLIES):
            plies()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(timed // GRAPH_PLIES):
            plies()
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / timed
        assert eng.error() == (0, -1)
        eng.close()
        del obs, eng
        torch.cuda.empty_cache()
        out[str(seed)] = dict(value=n / (ms / 1e3), ms_per_step=ms, warmup_plies=warm, timed_plies=timed)
    print(f"[bench] steady state: {out}", file=sys.stderr, flush=True)
    return out


def latency_bench(E, torch, eng, obs, samples=200):
    """Per-ply latency of the fused and the plain engine measured the same way:
    HIP events around each ply, one ply at a time (the fused ply as one direct
    launch, the plain ply as its four calls)."""
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def sample(fn):
        xs = []
        for i in range(samples + 4):
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            if i >= 4:
                xs.append(e0.elapsed_time(e1))
        return xs

    fused = sample(lambda: E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, num_legal=eng.num_legal,
                                                obs=obs))

    def plain_ply():
        eng.legal_mask()
        eng.sample()
        eng.encode()
        eng.step()
    plain = sample(plain_ply)
    assert eng.error() == (0, -1)
    out = dict(method="HIP events around each ply, one ply at a time", samples=samples,
               fused=dict(p50_ms=percentile(fused, 0.5), p99_ms=percentile(fused, 0.99),
                          value=n_rate(eng.n, fused)),
               plain=dict(p50_ms=percentile(plain, 0.5), p99_ms=percentile(plain, 0.99),
                          value=n_rate(eng.n, plain),
                          engine="plain per-call kernels (legal_mask, sample, encode_obs, step)"))
    print(f"[bench] latency: {out}", file=sys.stderr, flush=True)
    return out


def small_batch_bench(E, torch, sizes=(256, 4096), plies=192):
    """Small batches, where launches rather than bytes set the time: per-ply
    latency of the plain engine (four calls per ply), of single fused-ply
    launches and of fused plies replayed from 64-ply hipGraphs, each over the
    same plies of random play from fresh setups (no auto-reset), at every size
    in sizes, with the fused engine's tiling autotuned at that size.  Plain and
    direct fused plies are timed with HIP events around each ply; graph plies
    by the kernel's own per-ply timestamps."""
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for n in sizes:
        eng = E.Engine(n, SEED, K_BATTLELESS, MAX_MOVES, auto_reset=False)
        obs = eng.obs
        E.stratego_autotune(eng.ctx, obs, eng.mask, plies=8)
        G, S = E.stratego_get_tiling(eng.ctx)

        def each(fn):
            eng.reset()
            fn()                                   # warm-up ply (first launch of each kernel)
            eng.reset()
            xs = []
            for _ in range(plies):
                e0.record(stream)
                fn()
                e1.record(stream)
                e1.synchronize()
                xs.append(e0.elapsed_time(e1))
            return xs

        def plain_ply():
            eng.legal_mask()
            eng.sample()
            eng.encode()
            eng.step()
        plain = each(plain_ply)
        direct = each(lambda: E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, num_legal=eng.num_legal, obs=obs))
        ply_ns = torch.empty(GRAPH_PLIES, dtype=torch.int64, device="cuda")
        run = lambda: E.stratego_run_plies(eng.ctx, GRAPH_PLIES, mask=eng.mask, num_legal=eng.num_legal, obs=obs,
                                           use_graph=True, ply_ns=ply_ns)
        eng.reset()
        run()                                      # graph capture
        eng.reset()
        graph, graph_ms = [], 0.0
        for _ in range(plies // GRAPH_PLIES):
            e0.record(stream)
            run()
            e1.record(stream)
            e1.synchronize()
            graph_ms += e0.elapsed_time(e1)
            graph += [x / 1e6 for x in ply_ns.cpu().tolist()]
        assert eng.error() == (0, -1)
        eng.close()
        res = dict(plain=dict(p50_ms=percentile(plain, 0.5), p99_ms=percentile(plain, 0.99), value=n_rate(n, plain)),
                   fused_direct=dict(p50_ms=percentile(direct, 0.5), p99_ms=percentile(direct, 0.99),
                                     value=n_rate(n, direct)),
                   fused_graph=dict(p50_ms=percentile(graph, 0.5), p99_ms=percentile(graph, 0.99),
                                    ms_per_ply=graph_ms / (plies // GRAPH_PLIES * GRAPH_PLIES),
                                    value=n / (graph_ms / (plies // GRAPH_PLIES * GRAPH_PLIES) / 1e3)),
                   games_per_wg=G, lds_layout=S)
        out[str(n)] = res
        print(f"[bench] small batch n={n}: {res}", file=sys.stderr, flush=True)
    out["workload"] = (f"{plies} plies of random play from fresh setups (no auto-reset) per engine, "
                       f"mask + sample + both observations + step")
    return out


def n_rate(n, ms_list):
    return n / (sum(ms_list) / len(ms_list) / 1e3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6400, help="timed plies")
    ap.add_argument("--warmup", type=int, default=1024, help="untimed plies before timing")
    ap.add_argument("--games", type=int, default=GAMES)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-backfill-ms", type=float, default=5.0,
                    help="how long a serving request that does not fit lets later ones go ahead of it "
                         "(negative: strict arrival order)")
    ap.add_argument("--legs", default=None,
                    help="comma-separated subset of the extra legs to run: rollout_buffer, rules, policies, "
                         "acting, search, steady, small (default: all unless --no-extras)")
    ap.add_argument("--no-extras", "--no-history", dest="no_history", action="store_true",
                    help="skip the rollout-buffer, rules, policy, acting-player and search legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--tiling", default=None,
                    help="G,L: use this games-per-WG / LDS-layout tiling instead of autotuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: games shard across GPUs with no exchange "
              "step, so a run on N GPUs is N independent one-GPU runs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_07312_amd import engine as E

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n = args.games
    steps = max(1, args.steps)
    warmup = max(0, args.warmup)
    P, full, R = graph_split(steps)
    eng = E.Engine(n, SEED, K_BATTLELESS, MAX_MOVES, auto_reset=True)
    acts = torch.empty((P, n), dtype=torch.int16, device="cuda")
    done = torch.empty((P, n), dtype=torch.int8, device="cuda")
    outc = torch.empty((P, n), dtype=torch.int8, device="cuda")
    reas = torch.empty((P, n), dtype=torch.uint8, device="cuda")
    epl = torch.empty((P, n), dtype=torch.int16, device="cuda")
    ply_ns = torch.empty(P, dtype=torch.int64, device="cuda")
    obs = eng.obs

    def plies(k, use_graph, timed=False):
        E.stratego_run_plies(eng.ctx, k, mask=eng.mask, num_legal=eng.num_legal, actions=acts,
                             obs=obs, done=done, outcome=outc, reason=reas, ep_len=epl,
                             use_graph=use_graph, ply_ns=ply_ns[:k] if timed else None)

    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # warm-up: exactly `warmup` plies of the timed games (direct launches of
    # the same fused ply); long enough ones desynchronise the episodes
    for k0 in range(0, warmup, P):
        plies(min(P, warmup - k0), False)
    torch.cuda.synchronize()
    print(f"[bench] warm-up {warmup} plies done", file=sys.stderr, flush=True)

    # tiling: the autotuner times every tiling on the current states and
    # restores them afterwards, so its plies do not advance the timed games
    tune = []
    if args.tiling:
        g, s_ = (int(x) for x in args.tiling.split(","))
        E.stratego_set_tiling(eng.ctx, g, s_)
    elif not args.no_tune:
        tune = E.stratego_autotune(eng.ctx, obs, eng.mask, plies=8)
        print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    tuning_plies = 9 * len(tune)
    G, S = E.stratego_get_tiling(eng.ctx)
    plies(P, 2, True)                       # build the graphs for the chosen tiling
    if R:
        plies(R, 2, True)
    torch.cuda.synchronize()

    # timed region: exactly `steps` plies
    lat = []
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    per_launch = []
    for k in [P] * full + ([R] if R else []):
        plies(k, True, True)
        per_launch.append(ply_ns[:k].clone())
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    for t in per_launch:
        lat += [x / 1e6 for x in t.cpu().tolist()]
    assert len(lat) == steps
    assert eng.error() == (0, -1)
    ms_per_step = gpu_ms / steps
    value = n * steps / (gpu_ms / 1e3)
    kernel_ms = sum(lat) / len(lat)          # mean device duration of one ply kernel
    achieved = BYTES_PER_GAME_STEP * n / (ms_per_step / 1e3) / 1e9
    traffic = traffic_from_profile()
    print(f"[bench] timed {steps} plies: {gpu_ms:.1f} ms (wall {wall * 1e3:.1f} ms)",
          file=sys.stderr, flush=True)

    # store-only ceiling: PyTorch's fill of the same observation tensor (one
    # 16-byte store per thread, in address order)
    fill_ms = []
    for _ in range(6):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        obs.fill_(1)
        e1.record(stream)
        e1.synchronize()
        fill_ms.append(e0.elapsed_time(e1))
    fill_gbs = obs.numel() / (min(fill_ms[1:]) / 1e3) / 1e9
    store_ceiling = dict(kernel="torch fill_ of the observation tensor", GBs=fill_gbs,
                         fused_ply_frac=achieved / fill_gbs)
    print(f"[bench] store ceiling: {store_ceiling}", file=sys.stderr, flush=True)

    latency = None if args.no_plain else latency_bench(E, torch, eng, obs)
    eng.close()
    del obs, eng
    torch.cuda.empty_cache()
    serving = None if args.no_serving else serving_bench(E, torch, backfill_wait_s=args.serving_backfill_ms / 1e3)
    torch.cuda.empty_cache()
    legs = set(EXTRA_LEGS) if args.legs is None and not args.no_history else set()
    if args.legs:
        legs = set(x.strip() for x in args.legs.split(",") if x.strip())
        unknown = legs - set(EXTRA_LEGS)
        if unknown:
            raise SystemExit(f"unknown legs {sorted(unknown)}; known: {', '.join(EXTRA_LEGS)}")
    rollout_buffer = rollout_buffer_bench(E, torch, n) if "rollout_buffer" in legs else None
    torch.cuda.empty_cache()
    two_square = two_square_bench(E, torch, n) if "rules" in legs else None
    torch.cuda.empty_cache()
    policies = policy_bench(E, torch, n) if "policies" in legs else None
    torch.cuda.empty_cache()
    acting = acting_player_bench(E, torch, n) if "acting" in legs else None
    torch.cuda.empty_cache()
    search = search_bench(E, torch) if "search" in legs else None
    torch.cuda.empty_cache()
    steady = steady_state_bench(E, torch, G, S, n) if "steady" in legs else None
    torch.cuda.empty_cache()
    small = small_batch_bench(E, torch) if "small" in legs else None

    cpu = None if args.no_cpu_baseline else cpu_baseline()

    steady_reached = warmup >= 1000
    phase = ("after the episodes have desynchronised (at least 1000 plies of warm-up)" if steady_reached else
             f"plies {warmup}..{warmup + steps - 1} of the first episodes, before the 1000-ply steady state "
             "(see steady_state for that)")
    out = {
        "metric": "game steps/sec (mask+step+encode) at 65536 games; p50/p99 step latency",
        "value": value,
        "unit": "game steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic: uniform random setups and uniform random legal play (Philox4x32-10)",
        "config": {
            "workload": f"{n} games, fused persistent ply kernel (mask, sample, encode both "
                        f"players [2,488,10,10] uint8, step, auto-reset), {steps} timed plies from "
                        f"hipGraphs of {P} plies" + (f" and one of {R}" if R else "") + f"; {phase}",
            "games": n, "plies_per_graph": P, "k_battleless": K_BATTLELESS,
            "max_moves": MAX_MOVES, "seed": SEED, "games_per_wg": G, "lds_layout": S,
            "steady_state": steady_reached, "tuning_plies_on_restored_states": tuning_plies,
            "parallelism": "single GPU",
        },
        "p50_ms": percentile(lat, 0.5),
        "p99_ms": percentile(lat, 0.99),
        "latency_method": "device timestamps of each ply kernel (first wave start to last wave end)",
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per ply launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "algorithmic_bytes_per_launch": BYTES_PER_GAME_STEP * n,
            "kernel": f"k_ply<15, {1 if S == 1 else 2 if S == 7 else 0}> (fused ply)",
            "bytes_per_game_step": BYTES_PER_GAME_STEP,
            "kernel_ms_device_timestamps": kernel_ms,
        },
        "store_ceiling": store_ceiling,
        "latency_fused_vs_plain": latency,
        "steady_state": steady,
        "acting_player_only": acting,
        "serving": serving,
        "rollout_buffer": rollout_buffer,
        "competitive_rules": two_square,
        "policies": policies,
        "search_shaped": search,
        "small_batches": small,
        "autotune": [dict(games_per_wg=g, lds_layout=s, us_per_ply=u) for g, s, u in tune],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
