"""Fused plies over caller-owned records without allocation
(stratego_run_plies_static) give what stratego_run_plies gives on a context
holding the same records: every per-ply output and the final records,
bit-exact, on consecutive calls that reuse the static work counters, the
second with fewer games and plies."""
import pytest
import torch

from paper_2511_07312_amd import engine as E

pytestmark = pytest.mark.gpu

SEED = 4242
RULES = dict(k_battleless=100, max_moves=1000, auto_reset=True)


def _outputs(n, nplies, with_obs, fill):
    d = "cuda"
    out = dict(mask=torch.full((n, E.MASK_WORDS), fill, dtype=torch.int64, device=d),
               num_legal=torch.full((n,), fill, dtype=torch.int16, device=d),
               actions=torch.full((nplies * n,), fill, dtype=torch.int16, device=d),
               done=torch.full((nplies * n,), fill, dtype=torch.int8, device=d),
               outcome=torch.full((nplies * n,), fill, dtype=torch.int8, device=d),
               reason=torch.full((nplies * n,), fill, dtype=torch.uint8, device=d),
               ep_len=torch.full((nplies * n,), fill, dtype=torch.int16, device=d),
               obs=None)
    if with_obs:
        out["obs"] = torch.full((n, 2, E.NUM_CHANNELS, 10, 10), fill, dtype=torch.uint8, device=d)
    return out


def _compare(n, warm, nplies, with_obs):
    print(f"no-alloc plies: {n} games, {warm} warm-up plies, {nplies} plies, obs={with_obs}", flush=True)
    eng = E.Engine(n, SEED, **RULES)
    if warm:
        E.stratego_run_plies(eng.ctx, warm)   # mid-game states with uneven episodes
    start = eng.export()
    ref = _outputs(n, nplies, with_obs, 0x11)
    E.stratego_run_plies(eng.ctx, nplies, **ref)
    ref_states = eng.export()
    states = start.clone()
    got = _outputs(n, nplies, with_obs, 0x77)
    E.stratego_run_plies_static(states, nplies, SEED, **RULES, **got)
    torch.cuda.synchronize()
    for name, want in ref.items():
        if want is not None:
            assert torch.equal(got[name], want), f"{name} differs ({n} games, {nplies} plies)"
    assert torch.equal(states, ref_states), f"final records differ ({n} games)"
    assert eng.error() == (0, -1)
    eng.close()


def test_static_plies_match_the_context_engine_on_consecutive_calls():
    _compare(3000, 40, 5, True)
    _compare(777, 13, 3, True)      # fewer games and plies: the counters are reused
    _compare(777, 0, 4, False)      # observation-free plies from fresh setups


def test_static_plies_reject_bad_sizes():
    states = torch.zeros((4, E.RECORD_BYTES), dtype=torch.uint8, device="cuda")
    with pytest.raises(E.StrategoError):
        E.stratego_run_plies_static(states, E.STATIC_MAX_PLIES + 1, SEED, **RULES)
    with pytest.raises(E.StrategoError):
        E.stratego_run_plies_static(states, 1, SEED, games_per_wg=3, **RULES)
