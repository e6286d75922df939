"""Failure handling and resume, forced from the host: invalid configurations
and arguments, allocation failure at init, outputs poisoned before the
kernels (every byte must be written), and a serving rollout interrupted and
resumed from its exported records (the records are the checkpoint)."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2511_07312_amd import engine as E  # noqa: E402


def cpu(t):
    a = t.cpu().numpy()
    return a.view(np.uint64) if a.dtype == np.int64 and a.ndim == 2 and a.shape[-1] == 157 else a


@pytest.mark.parametrize("kw", [
    dict(num_games=0), dict(num_games=16, k_battleless=0), dict(num_games=16, max_moves=40000),
    dict(num_games=16, auto_reset=2), dict(num_games=16, games_per_wg=3), dict(num_games=16, lds_layout=8),
    dict(num_games=16, history_len=-1), dict(num_games=16, two_square=2), dict(num_games=16, sampler=2),
    dict(num_games=16, chasing=2), dict(num_games=16, acting_obs=3),
])
def test_invalid_configurations_are_refused(kw):
    args = dict(num_games=16, seed=1, k_battleless=100, max_moves=1000, auto_reset=False, game_id_base=0,
                games_per_wg=0, lds_layout=0, history_len=0, two_square=False, sampler=0, chasing=False,
                acting_obs=False)
    args.update(kw)
    cfg = E.StrategoConfig(args["num_games"], args["k_battleless"], args["max_moves"], args["auto_reset"],
                           args["seed"], args["game_id_base"], args["games_per_wg"], args["lds_layout"],
                           args["history_len"], int(args["two_square"]), args["sampler"], int(args["chasing"]),
                           int(args["acting_obs"]))
    import ctypes
    ctx = ctypes.c_void_p()
    rc = E.load_library().stratego_init(ctypes.byref(cfg), None, ctypes.byref(ctx))
    assert rc == E.E_INVAL and not ctx.value


def test_allocation_failure_at_init_is_reported():
    with pytest.raises(E.StrategoError) as err:
        E.Engine(4096, 1, history_len=1 << 20)       # 6.5 TB of ring
    assert err.value.code == E.E_NOMEM
    eng = E.Engine(64, 1)                             # the device is still usable
    eng.legal_mask()
    assert eng.error() == (0, -1)
    eng.close()


def test_null_arguments_are_refused():
    eng = E.Engine(64, 1)
    L = E.load_library()
    assert L.stratego_legal_mask(eng.ctx, None, None) == E.E_INVAL
    assert L.stratego_step(eng.ctx, None, None, None, None, None) == E.E_INVAL
    assert L.stratego_encode_obs(eng.ctx, None) == E.E_INVAL
    assert L.stratego_export_states(eng.ctx, None) == E.E_INVAL
    assert L.stratego_legal_mask(None, None, None) == E.E_INVAL
    assert L.stratego_run_plies(eng.ctx, -1, None, None, None, None, None, None, None, None, 0, None) == E.E_INVAL
    eng.close()


def test_poisoned_outputs_are_fully_written():
    """0xCD-filled outputs: after a fused ply and the plain calls every byte
    equals the oracle's, so none was left unwritten."""
    n, seed = 777, 6
    eng = E.Engine(n, seed, auto_reset=True)
    ref = O.OracleEngine(n, seed, auto_reset=True)
    for _ in range(20):
        E.stratego_run_plies(eng.ctx, 1)
        ref.ply(obs=False, mask=False)
    for buf in (eng.mask, eng.num_legal, eng.actions, eng.obs, eng.done, eng.outcome, eng.reason, eng.ep_len):
        buf.view(torch.uint8).fill_(0xCD)
    E.stratego_run_plies(eng.ctx, 1, mask=eng.mask, num_legal=eng.num_legal, actions=eng.actions,
                         obs=eng.obs, done=eng.done, outcome=eng.outcome, reason=eng.reason, ep_len=eng.ep_len)
    r = ref.ply(obs=True)
    for k in ("mask", "num_legal", "actions", "obs", "done", "outcome", "reason", "ep_len"):
        got = cpu(eng.mask if k == "mask" else getattr(eng, k))
        assert np.array_equal(got, r[k]), k
    eng.obs.fill_(0xCD)
    eng.mask.view(torch.uint8).fill_(0xCD)
    m, nl = ref.mask()
    assert np.array_equal(cpu(eng.legal_mask()[0]), m)
    assert np.array_equal(cpu(eng.encode()), ref.encode())
    recs = torch.full((n, E.RECORD_BYTES), 0xCD, dtype=torch.uint8, device="cuda")
    E.stratego_export_states(eng.ctx, recs)
    assert np.array_equal(cpu(recs), ref.export())
    eng.close()


def test_serving_rollout_interrupted_and_resumed_from_records():
    """A rollout of k plies equals a rollout of k1 plies followed, after the
    records were exported and re-admitted, by one of k - k1 plies."""
    n, seed, k, k1 = 900, 3, 37, 15
    ref = O.OracleEngine(n, seed)
    for _ in range(30):
        ref.ply(obs=False, mask=False)
    recs = torch.from_numpy(ref.export()).cuda()
    eng = E.Engine(2048, seed)
    whole = torch.zeros_like(recs)
    E.stratego_serve(eng.ctx, [(E.REQ_ROLLOUT, k, n, 0, 0.0)], recs, whole, realtime=False)
    part = torch.zeros_like(recs)
    E.stratego_serve(eng.ctx, [(E.REQ_ROLLOUT, k1, n, 0, 0.0)], recs, part, realtime=False)
    checkpoint = part.cpu().clone()                  # what a client would keep
    resumed = torch.zeros_like(recs)
    E.stratego_serve(eng.ctx, [(E.REQ_ROLLOUT, k - k1, n, 0, 0.0)], checkpoint.cuda(), resumed, realtime=False)
    assert torch.equal(resumed, whole)
    for _ in range(k):
        ref.ply(obs=False, mask=False)
    assert np.array_equal(cpu(whole), ref.export())
    assert eng.error() == (0, -1)
    eng.close()
