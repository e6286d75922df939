"""Magnet policy and search policy (sections 2.4-2.5, App. D.7) on the GPU vs the
oracle: legal lists, magnet probabilities, magnet sampling (plain and fused,
with and without the two-square rule) and the policy sampler bit-exact; the
single-precision search policy within the tolerance derived in the design
notes (relative 1e-4) of the oracle's double-precision one."""
import numpy as np
import pytest

import oracle as O

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


def played_records(n, seed, plies):
    ref = O.OracleEngine(n, seed, auto_reset=True)
    for _ in range(plies):
        ref.ply(obs=False, mask=False)
    return ref.export()


def positions(seed=0):
    from test_oracle_pins import random_position
    rng = np.random.default_rng(seed)
    sparse = [random_position(rng, int(rng.integers(1, 41)), int(rng.integers(1, 41))) for _ in range(300)]
    return np.concatenate([np.stack(sparse), played_records(700, 4, 60)])


@pytest.mark.parametrize("two_square", [False, True])
def test_fused_plies_with_the_magnet_sampler(two_square):
    n, seed = 1000, 21
    kw = dict(k_battleless=100, max_moves=400, auto_reset=True, two_square=two_square)
    eng = E.Engine(n, seed, sampler=E.SAMPLER_MAGNET, **kw)
    ref = O.OracleEngine(n, seed, sampler=O.SAMPLER_MAGNET, **kw)
    for ply in range(120):
        obs = ply % 30 == 0
        E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, num_legal=eng.num_legal, actions=eng.actions,
                             obs=eng.obs if obs else None, done=eng.done, outcome=eng.outcome,
                             reason=eng.reason, ep_len=eng.ep_len)
        r = ref.ply(obs=obs)
        assert_same(f"actions@{ply}", cpu(eng.actions), r["actions"])
        assert_same(f"mask@{ply}", cpu(eng.mask), r["mask"])
        if obs:
            assert_same(f"obs@{ply}", cpu(eng.obs), r["obs"])
        for k in ("done", "outcome", "reason", "ep_len"):
            assert_same(f"{k}@{ply}", cpu(getattr(eng, k)), r[k])
    assert_same("states", cpu(eng.export()), ref.export())
    # a graph of plies replays the same way
    E.stratego_run_plies(eng.ctx, 16, use_graph=True)
    for _ in range(16):
        ref.ply(obs=False, mask=False)
    assert_same("states after graph", cpu(eng.export()), ref.export())
    assert eng.error() == (0, -1)
    eng.close()


def test_plain_sampler_with_the_magnet_policy():
    recs = positions(1)
    n, seed = len(recs), 8
    eng = E.Engine(n, seed, sampler=E.SAMPLER_MAGNET)
    eng.load(torch.from_numpy(recs).cuda())
    ref = O.OracleEngine.from_records(recs, seed, sampler=O.SAMPLER_MAGNET)
    eng.legal_mask()
    eng.sample()
    m, nl = ref.mask()
    assert_same("mask", cpu(eng.mask), m)
    assert_same("magnet actions", cpu(eng.actions), ref.sample(m, nl))
    eng.close()


def test_legal_lists_and_magnet_probabilities():
    recs = positions(2)
    n = len(recs)
    eng = E.Engine(n, 3)
    eng.load(torch.from_numpy(recs).cuda())
    ref = O.OracleEngine.from_records(recs, 3)
    a, nl = eng.legal_list()
    wa, wnl = ref.legal_actions_list()
    assert_same("legal list", cpu(a), wa)
    assert_same("num_legal", cpu(nl), wnl)
    assert int(wnl.max()) <= 244
    assert_same("magnet", cpu(eng.magnet()).view(np.uint32), ref.magnet().view(np.uint32))
    eng.close()


def test_search_policy_and_policy_sampler():
    recs = positions(3)
    n, seed = len(recs), 5
    eng = E.Engine(n, seed)
    eng.load(torch.from_numpy(recs).cuda())
    ref = O.OracleEngine.from_records(recs, seed)
    _, nl = ref.legal_actions_list()
    rng = np.random.default_rng(9)
    valid = np.arange(256)[None, :] < nl[:, None]
    q = np.where(valid, rng.uniform(-1, 1, (n, 256)), 0).astype(np.float32)
    logits = rng.normal(0, 1.5, (n, 256))
    logits = np.where(valid, logits, -np.inf)
    logpi = logits - np.log(np.exp(logits).sum(axis=1, keepdims=True).clip(1e-300))
    logpi = np.where(valid, logpi, 0).astype(np.float32)
    for alpha, beta in ((0.002, 0.02), (0.3, 0.7), (1.0, 0.0)):
        got = cpu(eng.search_policy(torch.from_numpy(q).cuda(), torch.from_numpy(logpi).cuda(), alpha, beta))
        want = ref.mmd(q, logpi, alpha, beta)
        assert np.allclose(got, want, rtol=1e-4, atol=1e-12), np.abs(got - want).max()
        assert np.all(got[~valid] == 0)
        live = nl > 0
        assert np.allclose(got[live].sum(axis=1), 1.0, atol=1e-5)
        # the sampler takes its decision in single precision from the same inputs on both sides
        g = torch.from_numpy(got).cuda()
        assert_same(f"sampled ({alpha}, {beta})", cpu(eng.sample_policy(g)), ref.sample_policy(got))
    with pytest.raises(E.StrategoError):
        eng.search_policy(torch.from_numpy(q).cuda(), torch.from_numpy(logpi).cuda(), 0.0, 0.0)
    eng.close()
