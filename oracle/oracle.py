"""ctypes binding of the C oracle (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stratego_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

REC_BYTES = 1536
MAX_LEGAL = 256
SAMPLER_UNIFORM, SAMPLER_MAGNET = 0, 1
MASK_WORDS = 157
NCHAN = 488
OBS_BYTES = 2 * NCHAN * 100


def build(force=True):
    """Compile liboracle.so with gcc (plain C, OpenMP over games)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-shared", "-fPIC",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("k_battleless", ctypes.c_int32),
                ("max_moves", ctypes.c_int32), ("auto_reset", ctypes.c_int32),
                ("two_square", ctypes.c_int32), ("sampler", ctypes.c_int32), ("chasing", ctypes.c_int32),
                ("acting_obs", ctypes.c_int32), ("pad", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("STRATEGO_ORACLE_LIB")   # a test may point at a rebuilt copy
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.orc_state_bytes.restype = ctypes.c_size_t
        L.orc_batch_reset.argtypes = [P, ctypes.c_int, P, P]
        L.orc_batch_mask.argtypes = [P, ctypes.c_int, P, P, P]
        L.orc_batch_sample.argtypes = [P, ctypes.c_int, P, P, P, P]
        L.orc_batch_step.argtypes = [P, ctypes.c_int, P, P, P, P, P, P]
        L.orc_batch_step.restype = ctypes.c_int
        L.orc_batch_encode.argtypes = [P, ctypes.c_int, P, P]
        L.orc_batch_encode_subset.argtypes = [P, P, ctypes.c_int, P, P]
        L.orc_batch_export.argtypes = [P, ctypes.c_int, P]
        L.orc_batch_import.argtypes = [P, ctypes.c_int, P]
        L.orc_batch_resample.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_uint32, P]
        L.orc_batch_ply.argtypes = [P, ctypes.c_int, P, P, P, P, P, P, P, P, P]
        L.orc_legal_list.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
        L.orc_legal_list.restype = ctypes.c_int
        L.orc_has_legal_move.argtypes = [P, ctypes.c_int, ctypes.c_int]
        L.orc_has_legal_move.restype = ctypes.c_int
        L.orc_two_square_applies.argtypes = [P, P]
        L.orc_chase_applies.argtypes = [P, P]
        L.orc_chase_applies.restype = ctypes.c_int
        L.orc_batch_legal_list.argtypes = [P, ctypes.c_int, P, P, P]
        L.orc_batch_magnet.argtypes = [P, ctypes.c_int, P, P]
        L.orc_batch_mmd.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_double, ctypes.c_double, P]
        L.orc_batch_sample_policy.argtypes = [P, ctypes.c_int, P, P, P]
        L.orc_two_square_applies.restype = ctypes.c_int
        L.orc_terminal_check.argtypes = [P, P]
        L.orc_battle.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_battle.restype = ctypes.c_int
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_setup_types.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_int, P]
        L.orc_hidden_prob.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]
        L.orc_digest_blocks.argtypes = [P, ctypes.c_int64, ctypes.c_int64, P]
        L.orc_fnv1a64.argtypes = [P, ctypes.c_size_t]
        L.orc_fnv1a64.restype = ctypes.c_uint64
        L.orc_board_string.argtypes = [P, ctypes.c_char_p]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def battle(attacker_type, defender_type):
    """0 = attacker wins, 1 = defender wins, 2 = both removed."""
    return lib().orc_battle(int(attacker_type), int(defender_type))


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def setup_types(seed, game_id, episode, player):
    out = np.zeros(40, dtype=np.int32)
    lib().orc_setup_types(seed, game_id, episode, player, _p(out))
    return out


def num_threads():
    return int(lib().orc_num_threads())


def fnv1a64(buf):
    b = np.ascontiguousarray(buf).view(np.uint8)
    return int(lib().orc_fnv1a64(_p(b), b.nbytes))


def digest_blocks(buf, block):
    """Per-block digests (uint64) of a byte buffer cut into blocks of `block`
    bytes: sum of byte i times the SplitMix64 weight of i, modulo 2^64."""
    b = np.ascontiguousarray(buf).reshape(-1).view(np.uint8)
    assert b.size % block == 0
    out = np.zeros(b.size // block, dtype=np.uint64)
    lib().orc_digest_blocks(_p(b), b.size // block, int(block), _p(out))
    return out


def hidden_prob(engine, game, w, moved, t):
    num, den = ctypes.c_long(), ctypes.c_long()
    lib().orc_hidden_prob(engine._state_ptr(game), w, moved, t, ctypes.byref(num), ctypes.byref(den))
    return num.value, den.value


class OracleEngine:
    """N independent games advanced by the C oracle."""

    def __init__(self, n, seed, k_battleless=100, max_moves=1000, auto_reset=False,
                 game_ids=None, reset=True, two_square=False, sampler=SAMPLER_UNIFORM, chasing=False,
                 acting_obs=False):
        L = lib()
        self.n = int(n)
        self.sb = int(L.orc_state_bytes())
        self.states = np.zeros(self.n * self.sb, dtype=np.uint8)
        self.cfg = _Cfg(seed, k_battleless, max_moves, 1 if auto_reset else 0, 1 if two_square else 0,
                        int(sampler), 1 if chasing else 0, 1 if acting_obs else 0, 0)
        self.observers = 1 if acting_obs else 2
        if reset:
            self.reset(game_ids)

    def _cfgp(self):
        return ctypes.byref(self.cfg)

    def _state_ptr(self, i):
        return ctypes.c_void_p(self.states.ctypes.data + int(i) * self.sb)

    def reset(self, game_ids=None):
        if game_ids is None:
            game_ids = np.arange(self.n, dtype=np.uint32)
        ids = np.ascontiguousarray(game_ids, dtype=np.uint32)
        assert ids.shape == (self.n,)
        lib().orc_batch_reset(_p(self.states), self.n, self._cfgp(), _p(ids))

    def mask(self):
        m = np.zeros((self.n, MASK_WORDS), dtype=np.uint64)
        nl = np.zeros(self.n, dtype=np.int16)
        lib().orc_batch_mask(_p(self.states), self.n, self._cfgp(), _p(m), _p(nl))
        return m, nl

    def sample(self, mask, num_legal):
        a = np.zeros(self.n, dtype=np.int16)
        lib().orc_batch_sample(_p(self.states), self.n, self._cfgp(),
                               _p(np.ascontiguousarray(mask, dtype=np.uint64)),
                               _p(np.ascontiguousarray(num_legal, dtype=np.int16)), _p(a))
        return a

    def step(self, actions):
        act = np.ascontiguousarray(actions, dtype=np.int16)
        done = np.zeros(self.n, dtype=np.int8)
        outcome = np.zeros(self.n, dtype=np.int8)
        reason = np.zeros(self.n, dtype=np.uint8)
        ep_len = np.zeros(self.n, dtype=np.int16)
        bad = lib().orc_batch_step(_p(self.states), self.n, self._cfgp(), _p(act), _p(done),
                                   _p(outcome), _p(reason), _p(ep_len))
        return dict(done=done, outcome=outcome, reason=reason, ep_len=ep_len, first_bad=bad)

    def encode(self, idx=None):
        if idx is None:
            obs = np.zeros((self.n, self.observers, NCHAN, 10, 10), dtype=np.uint8)
            lib().orc_batch_encode(_p(self.states), self.n, self._cfgp(), _p(obs))
            return obs
        ix = np.ascontiguousarray(idx, dtype=np.int32)
        obs = np.zeros((len(ix), self.observers, NCHAN, 10, 10), dtype=np.uint8)
        lib().orc_batch_encode_subset(_p(self.states), _p(ix), len(ix), self._cfgp(), _p(obs))
        return obs

    def export(self):
        rec = np.zeros((self.n, REC_BYTES), dtype=np.uint8)
        lib().orc_batch_export(_p(self.states), self.n, _p(rec))
        return rec

    def load(self, records):
        rec = np.ascontiguousarray(records, dtype=np.uint8)
        assert rec.shape == (self.n, REC_BYTES)
        lib().orc_batch_import(_p(self.states), self.n, _p(rec))

    @classmethod
    def from_records(cls, records, seed, **kw):
        rec = np.ascontiguousarray(records, dtype=np.uint8)
        e = cls(rec.shape[0], seed, reset=False, **kw)
        e.load(rec)
        return e

    def resample(self, per, seed, game_id_base=0):
        """New engine holding per resamples of each game (game ids base + i*per + j)."""
        out = OracleEngine(self.n * per, seed, self.cfg.k_battleless, self.cfg.max_moves,
                           bool(self.cfg.auto_reset), reset=False, two_square=bool(self.cfg.two_square),
                           sampler=self.cfg.sampler, chasing=bool(self.cfg.chasing),
                           acting_obs=bool(self.cfg.acting_obs))
        lib().orc_batch_resample(_p(self.states), self.n, per, seed, game_id_base, _p(out.states))
        return out

    def ply(self, obs=True, mask=True, obs_out=None):
        """One fused ply; obs_out, if given, is a reused uint8 buffer for the
        observations (then returned as r["obs"])."""
        n = self.n
        if obs and obs_out is not None:
            assert obs_out.dtype == np.uint8 and obs_out.flags.c_contiguous
            assert obs_out.size == n * self.observers * NCHAN * 100
        r = dict(
            mask=np.zeros((n, MASK_WORDS), dtype=np.uint64) if mask else None,
            num_legal=np.zeros(n, dtype=np.int16),
            actions=np.zeros(n, dtype=np.int16),
            obs=(obs_out if obs_out is not None else np.zeros((n, self.observers, NCHAN, 10, 10), dtype=np.uint8))
            if obs else None,
            done=np.zeros(n, dtype=np.int8), outcome=np.zeros(n, dtype=np.int8),
            reason=np.zeros(n, dtype=np.uint8), ep_len=np.zeros(n, dtype=np.int16))
        lib().orc_batch_ply(_p(self.states), n, self._cfgp(), _p(r["mask"]), _p(r["num_legal"]),
                            _p(r["actions"]), _p(r["obs"]), _p(r["done"]), _p(r["outcome"]),
                            _p(r["reason"]), _p(r["ep_len"]))
        return r

    # -- policies over the legal list (sections 2.4-2.5, App. D.7) ---------------
    def legal_actions_list(self):
        """Legal actions of every game in ascending order, padded with -1."""
        a = np.zeros((self.n, MAX_LEGAL), dtype=np.int16)
        nl = np.zeros(self.n, dtype=np.int16)
        lib().orc_batch_legal_list(_p(self.states), self.n, self._cfgp(), _p(a), _p(nl))
        return a, nl

    def magnet(self):
        """The magnet policy over each game's legal list (float32)."""
        out = np.zeros((self.n, MAX_LEGAL), dtype=np.float32)
        lib().orc_batch_magnet(_p(self.states), self.n, self._cfgp(), _p(out))
        return out

    def mmd(self, q, logpi, alpha, beta):
        """The search policy over each legal list, in float64."""
        out = np.zeros((self.n, MAX_LEGAL), dtype=np.float64)
        lib().orc_batch_mmd(_p(self.states), self.n, self._cfgp(),
                            _p(np.ascontiguousarray(q, dtype=np.float32)),
                            _p(np.ascontiguousarray(logpi, dtype=np.float32)), float(alpha), float(beta),
                            _p(out))
        return out

    def sample_policy(self, probs):
        a = np.zeros(self.n, dtype=np.int16)
        lib().orc_batch_sample_policy(_p(self.states), self.n, self._cfgp(),
                                      _p(np.ascontiguousarray(probs, dtype=np.float32)), _p(a))
        return a

    def _rules(self, two_square, chasing):
        ts = self.cfg.two_square if two_square is None else int(bool(two_square))
        ch = self.cfg.chasing if chasing is None else int(bool(chasing))
        return ts | (ch << 1)

    def legal_list(self, game, player, two_square=None, chasing=None):
        legal = np.zeros(10000, dtype=np.uint8)
        n = lib().orc_legal_list(self._state_ptr(game), player, self._rules(two_square, chasing), _p(legal))
        return n, legal

    def has_legal_move(self, game, player, two_square=None, chasing=None):
        return bool(lib().orc_has_legal_move(self._state_ptr(game), player, self._rules(two_square, chasing)))

    def chase_applies(self, game):
        """The continuous-chasing rule removes a move of the acting player."""
        return bool(lib().orc_chase_applies(self._state_ptr(game), self._cfgp()))

    def two_square_applies(self, game):
        """App. B.1 ComputeTwoSquareRuleApplies for one game."""
        return bool(lib().orc_two_square_applies(self._state_ptr(game), self._cfgp()))

    def terminal_check(self, game):
        lib().orc_terminal_check(self._state_ptr(game), self._cfgp())

    def board_string(self, game):
        buf = ctypes.create_string_buffer(400)
        lib().orc_board_string(self._state_ptr(game), buf)
        return buf.value.decode()
