"""Python binding of libstratego.so (argument marshalling only).

Every function mirrors the C call of the same name in include/stratego.h.
Device buffers are torch tensors on the GPU; a context runs on torch's
current stream at the time it is created.  All game computation happens in the
library's kernels: the library is loaded on first use, a missing library
raises an error there, and there is no CPU fallback.
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libstratego.so")

OK = 0
E_INVAL = -1
E_NOMEM = -2
E_HIP = -3
E_ILLEGAL_ACTION = -4
E_BAD_STATE = -5
E_RANGE = -6
NUM_CHANNELS = 488
MASK_WORDS = 157
RECORD_BYTES = 1536
OBS_BYTES_PER_GAME = 97600
HISTORY_BYTES_PER_GAME_STEP = 1544
MAX_LEGAL = 256
STATIC_MAX_PLIES = 4096
SAMPLER_UNIFORM = 0
SAMPLER_MAGNET = 1

FUNCTIONS = [
    "stratego_init", "stratego_reset", "stratego_legal_mask", "stratego_sample_actions",
    "stratego_step", "stratego_encode_obs", "stratego_export_states", "stratego_run_plies",
    "stratego_run_plies_slots", "stratego_reset_resampled", "stratego_autotune",
    "stratego_get_tiling", "stratego_set_tiling", "stratego_get_error", "stratego_current_step",
    "stratego_destroy", "stratego_strerror", "stratego_serve", "stratego_history_window",
    "stratego_history_legal_mask", "stratego_history_encode_obs", "stratego_history_info",
    "stratego_history_export", "stratego_legal_list", "stratego_magnet_policy",
    "stratego_search_policy", "stratego_sample_policy", "stratego_board_strings",
    "stratego_run_plies_static",
]
REQ_STEP = 0
REQ_ROLLOUT = 1


class StrategoConfig(ctypes.Structure):
    _fields_ = [("num_games", ctypes.c_int32), ("k_battleless", ctypes.c_int32),
                ("max_moves", ctypes.c_int32), ("auto_reset", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("game_id_base", ctypes.c_uint32),
                ("games_per_wg", ctypes.c_int32), ("lds_layout", ctypes.c_int32),
                ("history_len", ctypes.c_int32), ("two_square_rule", ctypes.c_int32),
                ("sampler", ctypes.c_int32), ("chasing_rule", ctypes.c_int32),
                ("acting_obs_only", ctypes.c_int32)]


class HistoryOutputs(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in (
        "acting_player", "played_action", "num_moves", "moves_since_attack", "reward_pl0",
        "terminated_since", "has_legal_movement", "flag_captured", "is_unknown", "piece_onehot",
        "two_square_applies", "chase_applies")]


# dtype and elements per listed game of each history_info output
HISTORY_INFO = {
    "acting_player": (torch.int8, 1), "played_action": (torch.int16, 1),
    "num_moves": (torch.int32, 1), "moves_since_attack": (torch.int32, 1),
    "reward_pl0": (torch.int8, 1), "terminated_since": (torch.int32, 1),
    "has_legal_movement": (torch.uint8, 1), "flag_captured": (torch.uint8, 1),
    "is_unknown": (torch.uint8, 100), "piece_onehot": (torch.uint8, 2400),
    "two_square_applies": (torch.uint8, 1), "chase_applies": (torch.uint8, 1),
}


class TuneEntry(ctypes.Structure):
    _fields_ = [("games_per_wg", ctypes.c_int32), ("lds_layout", ctypes.c_int32),
                ("us_per_ply", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("plies", ctypes.c_int32), ("num_games", ctypes.c_int32),
                ("first", ctypes.c_int32), ("arrival_s", ctypes.c_double)]


class RequestResult(ctypes.Structure):
    _fields_ = [("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("game_steps", ctypes.c_int64),
                ("iterations", ctypes.c_int32), ("peak_active_games", ctypes.c_int32),
                ("peak_reserved_bytes", ctypes.c_int64), ("budget_bytes", ctypes.c_int64),
                ("gpu_busy_s", ctypes.c_double), ("gpu_span_s", ctypes.c_double)]


class StrategoError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


_lib = None


def load_library(path=LIB_PATH):
    """Load libstratego.so (without touching the GPU)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() first")
    L = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.stratego_init.argtypes = [ctypes.POINTER(StrategoConfig), P, ctypes.POINTER(P)]
    L.stratego_reset.argtypes = [P, P, I32, P]
    L.stratego_legal_mask.argtypes = [P, P, P]
    L.stratego_sample_actions.argtypes = [P, P, P, P]
    L.stratego_step.argtypes = [P, P, P, P, P, P]
    L.stratego_encode_obs.argtypes = [P, P]
    L.stratego_export_states.argtypes = [P, P]
    L.stratego_run_plies.argtypes = [P, I32, P, P, P, P, P, P, P, P, I32, P]
    L.stratego_run_plies_slots.argtypes = [P, P, I32, I32, P, P, P, P, P, P, P]
    L.stratego_reset_resampled.argtypes = [P, P, I32, I32, ctypes.c_uint32]
    L.stratego_autotune.argtypes = [P, P, P, I32, ctypes.POINTER(TuneEntry), I32,
                                    ctypes.POINTER(I32)]
    L.stratego_get_tiling.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    L.stratego_set_tiling.argtypes = [P, I32, I32]
    L.stratego_get_error.argtypes = [P, ctypes.POINTER(I32)]
    L.stratego_current_step.argtypes = [P, ctypes.POINTER(I64)]
    L.stratego_destroy.argtypes = [P]
    L.stratego_serve.argtypes = [P, ctypes.POINTER(Request), I32, P, P, P, I32, I64, I32,
                                 ctypes.c_double, ctypes.POINTER(RequestResult),
                                 ctypes.POINTER(ServeStats)]
    L.stratego_history_window.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    L.stratego_history_legal_mask.argtypes = [P, I64, P, I32, P, P]
    L.stratego_history_encode_obs.argtypes = [P, I64, P, I32, P]
    L.stratego_history_info.argtypes = [P, I64, P, I32, ctypes.POINTER(HistoryOutputs)]
    L.stratego_history_export.argtypes = [P, I64, P, I32, P]
    L.stratego_legal_list.argtypes = [P, P, P]
    L.stratego_magnet_policy.argtypes = [P, P]
    L.stratego_search_policy.argtypes = [P, P, P, ctypes.c_float, ctypes.c_float, P]
    L.stratego_sample_policy.argtypes = [P, P, P]
    L.stratego_board_strings.argtypes = [P, I64, P, I32, ctypes.c_char_p]
    L.stratego_run_plies_static.argtypes = [ctypes.POINTER(StrategoConfig), P, P, I32, P, P, P, P, P, P, P, P]
    L.stratego_strerror.argtypes = [ctypes.c_int]
    L.stratego_strerror.restype = ctypes.c_char_p
    for f in FUNCTIONS:
        if f != "stratego_strerror":
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def strerror(code):
    return load_library().stratego_strerror(int(code)).decode()


def _check(rc, what):
    if rc != OK:
        raise StrategoError(rc, what)


def _ptr(t, dtype=None, numel=None, name="buffer"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ C-ABI mirrors
def stratego_init(num_games, seed, k_battleless=100, max_moves=4000, auto_reset=False,
                  game_id_base=0, games_per_wg=0, lds_layout=0, history_len=0, two_square=False,
                  sampler=SAMPLER_UNIFORM, chasing=False, acting_obs=False):
    cfg = StrategoConfig(int(num_games), int(k_battleless), int(max_moves), int(bool(auto_reset)),
                         int(seed), int(game_id_base), int(games_per_wg), int(lds_layout),
                         int(history_len), int(bool(two_square)), int(sampler), int(bool(chasing)),
                         int(bool(acting_obs)))
    ctx = ctypes.c_void_p()
    _check(load_library().stratego_init(ctypes.byref(cfg), _stream(), ctypes.byref(ctx)),
           "stratego_init")
    _ctx_games[ctx.value] = int(num_games)
    _ctx_obs[ctx.value] = OBS_BYTES_PER_GAME // 2 if acting_obs else OBS_BYTES_PER_GAME
    return ctx


def stratego_reset(ctx, slots=None, n=None, states=None):
    if n is None:
        n = slots.numel() if slots is not None else (states.shape[0] if states is not None else None)
    _check(load_library().stratego_reset(ctx, _ptr(slots, torch.int32, n, "slots"), int(n),
                                         _ptr(states, torch.uint8, n * RECORD_BYTES, "states")),
           "stratego_reset")


def stratego_legal_mask(ctx, mask, num_legal=None):
    n = _num_games(ctx)
    _check(load_library().stratego_legal_mask(ctx, _ptr(mask, torch.int64, n and n * MASK_WORDS, "mask"),
                                              _ptr(num_legal, torch.int16, n, "num_legal")),
           "stratego_legal_mask")


def stratego_sample_actions(ctx, mask, num_legal, actions):
    n = _num_games(ctx)
    _check(load_library().stratego_sample_actions(
        ctx, _ptr(mask, torch.int64, n and n * MASK_WORDS, "mask"),
        _ptr(num_legal, torch.int16, n, "num_legal"),
        _ptr(actions, torch.int16, n, "actions")), "stratego_sample_actions")


def stratego_step(ctx, actions, done=None, outcome=None, reason=None, ep_len=None):
    n = _num_games(ctx)
    _check(load_library().stratego_step(
        ctx, _ptr(actions, torch.int16, n, "actions"), _ptr(done, torch.int8, n, "done"),
        _ptr(outcome, torch.int8, n, "outcome"), _ptr(reason, torch.uint8, n, "reason"),
        _ptr(ep_len, torch.int16, n, "ep_len")), "stratego_step")


def stratego_encode_obs(ctx, obs):
    n = _num_games(ctx)
    _check(load_library().stratego_encode_obs(
        ctx, _ptr(obs, torch.uint8, n and n * obs_bytes_per_game(ctx), "obs")), "stratego_encode_obs")


def stratego_export_states(ctx, states):
    n = _num_games(ctx)
    _check(load_library().stratego_export_states(
        ctx, _ptr(states, torch.uint8, n and n * RECORD_BYTES, "states")), "stratego_export_states")


def _listed(games, count):
    if games is None:
        if count is None:
            raise ValueError("count is required when games is None")
        return int(count)
    return int(games.numel()) if count is None else int(count)


def stratego_history_window(ctx):
    """Returns (oldest, current) time steps of the rollout buffer."""
    lo, cur = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().stratego_history_window(ctx, ctypes.byref(lo), ctypes.byref(cur)),
           "stratego_history_window")
    return lo.value, cur.value


def stratego_history_legal_mask(ctx, t, mask=None, num_legal=None, games=None, count=None):
    m = _listed(games, count)
    _check(load_library().stratego_history_legal_mask(
        ctx, int(t), _ptr(games, torch.int32, m, "games"), m,
        _ptr(mask, torch.int64, m * MASK_WORDS, "mask"), _ptr(num_legal, torch.int16, m, "num_legal")),
        "stratego_history_legal_mask")


def stratego_history_encode_obs(ctx, t, obs, games=None, count=None):
    m = _listed(games, count)
    _check(load_library().stratego_history_encode_obs(
        ctx, int(t), _ptr(games, torch.int32, m, "games"), m,
        _ptr(obs, torch.uint8, m * obs_bytes_per_game(ctx), "obs")), "stratego_history_encode_obs")


def stratego_history_info(ctx, t, games=None, count=None, **outputs):
    """outputs: any of the HISTORY_INFO names mapped to GPU tensors."""
    m = _listed(games, count)
    out = HistoryOutputs()
    for name, tensor in outputs.items():
        if name not in HISTORY_INFO:
            raise TypeError(f"unknown history output {name}")
        dtype, per = HISTORY_INFO[name]
        setattr(out, name, _ptr(tensor, dtype, m * per, name))
    _check(load_library().stratego_history_info(ctx, int(t), _ptr(games, torch.int32, m, "games"), m,
                                                ctypes.byref(out)), "stratego_history_info")


def stratego_history_export(ctx, t, states, games=None, count=None):
    m = _listed(games, count)
    _check(load_library().stratego_history_export(
        ctx, int(t), _ptr(games, torch.int32, m, "games"), m,
        _ptr(states, torch.uint8, m * RECORD_BYTES, "states")), "stratego_history_export")


BOARD_STRING_BYTES = 301


def stratego_board_strings(ctx, t, games=None, count=None):
    """BoardStrs of App. B: a text picture of each listed game's board at t."""
    m = _listed(games, count)
    if m == 0:
        return []
    buf = ctypes.create_string_buffer(m * BOARD_STRING_BYTES)
    _check(load_library().stratego_board_strings(ctx, int(t), _ptr(games, torch.int32, m, "games"), m, buf),
           "stratego_board_strings")
    raw = buf.raw
    return [raw[i * BOARD_STRING_BYTES:(i + 1) * BOARD_STRING_BYTES].split(b"\0", 1)[0].decode()
            for i in range(m)]


def stratego_legal_list(ctx, actions, num_legal=None):
    n = _num_games(ctx)
    _check(load_library().stratego_legal_list(
        ctx, _ptr(actions, torch.int16, n and n * MAX_LEGAL, "actions"),
        _ptr(num_legal, torch.int16, n, "num_legal")), "stratego_legal_list")


def stratego_magnet_policy(ctx, probs):
    n = _num_games(ctx)
    _check(load_library().stratego_magnet_policy(ctx, _ptr(probs, torch.float32, n and n * MAX_LEGAL, "probs")),
           "stratego_magnet_policy")


def stratego_search_policy(ctx, q, logpi, alpha, beta, probs):
    n = _num_games(ctx)
    per = n and n * MAX_LEGAL
    _check(load_library().stratego_search_policy(
        ctx, _ptr(q, torch.float32, per, "q"), _ptr(logpi, torch.float32, per, "logpi"), float(alpha),
        float(beta), _ptr(probs, torch.float32, per, "probs")), "stratego_search_policy")


def stratego_sample_policy(ctx, probs, actions):
    n = _num_games(ctx)
    _check(load_library().stratego_sample_policy(
        ctx, _ptr(probs, torch.float32, n and n * MAX_LEGAL, "probs"), _ptr(actions, torch.int16, n, "actions")),
        "stratego_sample_policy")


def _num_games(ctx):
    return _ctx_games.get(ctx.value)


def obs_bytes_per_game(ctx):
    """97,600 (both players) or 48,800 (acting player only)."""
    return _ctx_obs.get(ctx.value, OBS_BYTES_PER_GAME)


_ctx_games = {}
_ctx_obs = {}


def stratego_run_plies(ctx, nplies, mask=None, num_legal=None, actions=None, obs=None, done=None,
                       outcome=None, reason=None, ep_len=None, use_graph=False, ply_ns=None):
    """use_graph: False/0 direct launches, True/1 replay a captured graph, 2
    build and upload the graph only (nothing runs)."""
    n = _num_games(ctx)
    per = None if n is None else int(nplies) * n
    _check(load_library().stratego_run_plies(
        ctx, int(nplies), _ptr(mask, torch.int64, n and n * MASK_WORDS, "mask"),
        _ptr(num_legal, torch.int16, n, "num_legal"), _ptr(actions, torch.int16, per, "actions"),
        _ptr(obs, torch.uint8, n and n * obs_bytes_per_game(ctx), "obs"),
        _ptr(done, torch.int8, per, "done"), _ptr(outcome, torch.int8, per, "outcome"),
        _ptr(reason, torch.uint8, per, "reason"), _ptr(ep_len, torch.int16, per, "ep_len"),
        int(use_graph), _ptr(ply_ns, torch.int64, int(nplies), "ply_ns")),
        "stratego_run_plies")


def stratego_run_plies_static(states, nplies, seed, k_battleless=100, max_moves=4000, auto_reset=False,
                              games_per_wg=0, lds_layout=0, two_square=False, sampler=SAMPLER_UNIFORM,
                              chasing=False, acting_obs=False, mask=None, num_legal=None, actions=None,
                              obs=None, done=None, outcome=None, reason=None, ep_len=None):
    """Fused plies over caller-owned records (uint8 [N, 1536] on the GPU), on
    torch's current stream, without allocation or a context."""
    n = int(states.shape[0])
    per = int(nplies) * n
    cfg = StrategoConfig(n, int(k_battleless), int(max_moves), int(bool(auto_reset)), int(seed), 0,
                         int(games_per_wg), int(lds_layout), 0, int(bool(two_square)), int(sampler),
                         int(bool(chasing)), int(bool(acting_obs)))
    obs_bytes = OBS_BYTES_PER_GAME // 2 if acting_obs else OBS_BYTES_PER_GAME
    _check(load_library().stratego_run_plies_static(
        ctypes.byref(cfg), _stream(), _ptr(states, torch.uint8, n * RECORD_BYTES, "states"), int(nplies),
        _ptr(mask, torch.int64, n * MASK_WORDS, "mask"), _ptr(num_legal, torch.int16, n, "num_legal"),
        _ptr(actions, torch.int16, per, "actions"), _ptr(obs, torch.uint8, n * obs_bytes, "obs"),
        _ptr(done, torch.int8, per, "done"), _ptr(outcome, torch.int8, per, "outcome"),
        _ptr(reason, torch.uint8, per, "reason"), _ptr(ep_len, torch.int16, per, "ep_len")),
        "stratego_run_plies_static")


def stratego_run_plies_slots(ctx, slots, nplies, mask=None, actions=None, obs=None, done=None,
                             outcome=None, reason=None, ep_len=None):
    m = int(slots.numel())
    per = int(nplies) * m
    _check(load_library().stratego_run_plies_slots(
        ctx, _ptr(slots, torch.int32, m, "slots"), m, int(nplies),
        _ptr(mask, torch.int64, m * MASK_WORDS, "mask"), _ptr(actions, torch.int16, per, "actions"),
        _ptr(obs, torch.uint8, m * obs_bytes_per_game(ctx), "obs"), _ptr(done, torch.int8, per, "done"),
        _ptr(outcome, torch.int8, per, "outcome"), _ptr(reason, torch.uint8, per, "reason"),
        _ptr(ep_len, torch.int16, per, "ep_len")), "stratego_run_plies_slots")


def stratego_reset_resampled(ctx, src_states, per, game_id_base=0):
    nsrc = src_states.shape[0]
    _check(load_library().stratego_reset_resampled(
        ctx, _ptr(src_states, torch.uint8, nsrc * RECORD_BYTES, "src_states"), int(nsrc), int(per),
        int(game_id_base)), "stratego_reset_resampled")


def stratego_autotune(ctx, obs, mask, plies=3, max_entries=64):
    rep = (TuneEntry * max_entries)()
    n = ctypes.c_int32()
    _check(load_library().stratego_autotune(ctx, _ptr(obs, torch.uint8, None, "obs"),
                                            _ptr(mask, torch.int64, None, "mask"), int(plies), rep,
                                            max_entries, ctypes.byref(n)), "stratego_autotune")
    return [(rep[i].games_per_wg, rep[i].lds_layout, rep[i].us_per_ply) for i in range(n.value)]


def stratego_serve(ctx, requests, in_states, out_states, obs_out=None, obs_by_slot=False,
                   mem_budget_bytes=0, realtime=True, backfill_wait_s=-1.0):
    """requests: sequence of (kind, plies, num_games, first, arrival_s).
    backfill_wait_s < 0: strict arrival order; otherwise how long a request
    that does not fit lets later ones go ahead of it.
    Returns (list of (admit_s, done_s), stats dict)."""
    nreq = len(requests)
    reqs = (Request * max(nreq, 1))()
    total = 0
    for r, (kind, plies, b, first, arr) in enumerate(requests):
        reqs[r] = Request(int(kind), int(plies), int(b), int(first), float(arr))
        total = max(total, int(first) + int(b))
    res = (RequestResult * max(nreq, 1))()
    st = ServeStats()
    obs_rows = None if obs_out is None or obs_by_slot else total * obs_bytes_per_game(ctx)
    _check(load_library().stratego_serve(
        ctx, reqs, nreq, _ptr(in_states, torch.uint8, total * RECORD_BYTES, "in_states"),
        _ptr(out_states, torch.uint8, total * RECORD_BYTES, "out_states"),
        _ptr(obs_out, torch.uint8, obs_rows, "obs_out"), int(bool(obs_by_slot)),
        int(mem_budget_bytes), int(bool(realtime)), float(backfill_wait_s), res, ctypes.byref(st)),
        "stratego_serve")
    stats = {k: getattr(st, k) for k, _ in ServeStats._fields_}
    return [(res[r].admit_s, res[r].done_s) for r in range(nreq)], stats


def stratego_get_tiling(ctx):
    g, s = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().stratego_get_tiling(ctx, ctypes.byref(g), ctypes.byref(s)),
           "stratego_get_tiling")
    return g.value, s.value


def stratego_set_tiling(ctx, games_per_wg, lds_layout):
    _check(load_library().stratego_set_tiling(ctx, int(games_per_wg), int(lds_layout)),
           "stratego_set_tiling")


def stratego_get_error(ctx):
    slot = ctypes.c_int32()
    rc = load_library().stratego_get_error(ctx, ctypes.byref(slot))
    return rc, slot.value


def stratego_current_step(ctx):
    v = ctypes.c_int64()
    _check(load_library().stratego_current_step(ctx, ctypes.byref(v)), "stratego_current_step")
    return v.value


def stratego_destroy(ctx):
    _check(load_library().stratego_destroy(ctx), "stratego_destroy")
    _ctx_games.pop(ctx.value, None)
    _ctx_obs.pop(ctx.value, None)


# ------------------------------------------------------------------ convenience
class Engine:
    """N games on the current GPU with preallocated output tensors."""

    def __init__(self, num_games, seed, k_battleless=100, max_moves=1000, auto_reset=False,
                 game_id_base=0, games_per_wg=0, lds_layout=0, history_len=0, two_square=False,
                 sampler=SAMPLER_UNIFORM, chasing=False, acting_obs=False, device="cuda"):
        self.n = int(num_games)
        self.device = torch.device(device)
        self.ctx = stratego_init(num_games, seed, k_battleless, max_moves, auto_reset,
                                 game_id_base, games_per_wg, lds_layout, history_len, two_square, sampler,
                                 chasing, acting_obs)
        self.observers = 1 if acting_obs else 2
        n, d = self.n, self.device
        self.mask = torch.empty((n, MASK_WORDS), dtype=torch.int64, device=d)
        self.num_legal = torch.empty(n, dtype=torch.int16, device=d)
        self.actions = torch.empty(n, dtype=torch.int16, device=d)
        self.done = torch.empty(n, dtype=torch.int8, device=d)
        self.outcome = torch.empty(n, dtype=torch.int8, device=d)
        self.reason = torch.empty(n, dtype=torch.uint8, device=d)
        self.ep_len = torch.empty(n, dtype=torch.int16, device=d)
        self._obs = None

    @property
    def obs(self):
        if self._obs is None:
            self._obs = torch.empty((self.n, self.observers, NUM_CHANNELS, 10, 10), dtype=torch.uint8,
                                    device=self.device)
        return self._obs

    def legal_mask(self):
        stratego_legal_mask(self.ctx, self.mask, self.num_legal)
        return self.mask, self.num_legal

    def sample(self):
        stratego_sample_actions(self.ctx, self.mask, self.num_legal, self.actions)
        return self.actions

    def step(self, actions=None):
        stratego_step(self.ctx, self.actions if actions is None else actions, self.done,
                      self.outcome, self.reason, self.ep_len)
        return self.done, self.outcome, self.reason, self.ep_len

    def encode(self):
        stratego_encode_obs(self.ctx, self.obs)
        return self.obs

    def export(self):
        out = torch.empty((self.n, RECORD_BYTES), dtype=torch.uint8, device=self.device)
        stratego_export_states(self.ctx, out)
        return out

    def load(self, records, slots=None):
        stratego_reset(self.ctx, slots, records.shape[0], records)

    def reset(self, slots=None, n=None):
        stratego_reset(self.ctx, slots, self.n if n is None and slots is None else n, None)

    def error(self):
        return stratego_get_error(self.ctx)

    # policies over legal lists (sections 2.4-2.5, App. D.7)
    def legal_list(self):
        a = torch.empty((self.n, MAX_LEGAL), dtype=torch.int16, device=self.device)
        nl = torch.empty(self.n, dtype=torch.int16, device=self.device)
        stratego_legal_list(self.ctx, a, nl)
        return a, nl

    def magnet(self):
        p = torch.empty((self.n, MAX_LEGAL), dtype=torch.float32, device=self.device)
        stratego_magnet_policy(self.ctx, p)
        return p

    def search_policy(self, q, logpi, alpha=0.002, beta=0.02):
        p = torch.empty((self.n, MAX_LEGAL), dtype=torch.float32, device=self.device)
        stratego_search_policy(self.ctx, q, logpi, alpha, beta, p)
        return p

    def sample_policy(self, probs):
        a = torch.empty(self.n, dtype=torch.int16, device=self.device)
        stratego_sample_policy(self.ctx, probs, a)
        return a

    # rollout-buffer queries (App. B.1)
    def window(self):
        return stratego_history_window(self.ctx)

    def _list(self, games):
        return self.n if games is None else int(games.numel())

    def mask_at(self, t, games=None):
        m = self._list(games)
        mask = torch.empty((m, MASK_WORDS), dtype=torch.int64, device=self.device)
        nl = torch.empty(m, dtype=torch.int16, device=self.device)
        stratego_history_legal_mask(self.ctx, t, mask, nl, games, m)
        return mask, nl

    def obs_at(self, t, games=None, out=None):
        m = self._list(games)
        if out is None:
            out = torch.empty((m, self.observers, NUM_CHANNELS, 10, 10), dtype=torch.uint8, device=self.device)
        stratego_history_encode_obs(self.ctx, t, out, games, m)
        return out

    def info_at(self, t, games=None):
        m = self._list(games)
        outs = {name: torch.empty((m, per) if per > 1 else (m,), dtype=dtype, device=self.device)
                for name, (dtype, per) in HISTORY_INFO.items()}
        stratego_history_info(self.ctx, t, games, m, **outs)
        outs["piece_onehot"] = outs["piece_onehot"].view(m, 24, 100)
        return outs

    def export_at(self, t, games=None):
        m = self._list(games)
        out = torch.empty((m, RECORD_BYTES), dtype=torch.uint8, device=self.device)
        stratego_history_export(self.ctx, t, out, games, m)
        return out

    def board_strs(self, t=None, games=None):
        """BoardStrs: one text picture per game at time step t (default: now)."""
        return stratego_board_strings(self.ctx, self.window()[1] if t is None else t, games, self._list(games))

    def close(self):
        if self.ctx is not None:
            stratego_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
