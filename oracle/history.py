"""Rollout-buffer oracle (test infrastructure only).

App. B.1 describes a simulator that is also the rollout buffer: it keeps a
circular history of recent time steps and recomputes past legal-action masks
and information states on demand.  This module states that behaviour plainly:
it keeps, for each whole-batch ply of an ``OracleEngine``, the canonical
records the ply started from and the ply's outputs, and answers every query by
re-loading those records into a fresh oracle engine.  Time step t is the number
of whole-batch plies applied so far; ply t maps the states at t to those at
t + 1; the window is [max(0, T - H), T] with T the current time step.

The per-game scalar and per-square queries (App. B.1's table of historical
queries) are written out from their definitions on the record bytes.
"""
import numpy as np

from .oracle import OracleEngine

# canonical record offsets (header, board, pieces)
_PLY, _BATTLELESS, _DONE = 8, 12, 17
_BOARD, _PIECES = 64, 256
_REASON_FLAG = 1


class WindowError(IndexError):
    pass


def _u32(rec, off):
    return int(rec[off]) | int(rec[off + 1]) << 8 | int(rec[off + 2]) << 16 | int(rec[off + 3]) << 24


class OracleRolloutBuffer:
    """Records the plies of ``engine`` in a ring of H time steps."""

    def __init__(self, engine, history_len):
        self.e = engine
        self.H = int(history_len)
        self.t = 0
        self.rows = {}   # t -> dict(records, actions, done, outcome, reason, ep_len)

    # -- recording ---------------------------------------------------------
    def _push(self, records, actions, out):
        if self.H > 0:
            self.rows[self.t] = dict(records=records, actions=np.asarray(actions, dtype=np.int16).copy(),
                                     done=out["done"].copy(), outcome=out["outcome"].copy(),
                                     reason=out["reason"].copy(), ep_len=out["ep_len"].copy())
            self.rows.pop(self.t - self.H, None)
        self.t += 1

    def ply(self, obs=True, mask=True):
        """One fused ply (mask, sample, encode, step) of every game."""
        rec = self.e.export()
        r = self.e.ply(obs=obs, mask=mask)
        self._push(rec, r["actions"], r)
        return r

    def step(self, actions):
        """ApplyActions with caller actions."""
        rec = self.e.export()
        r = self.e.step(actions)
        self._push(rec, actions, r)
        return r

    # -- queries -----------------------------------------------------------
    def window(self):
        return max(0, self.t - self.H), self.t

    def _check(self, t):
        lo, hi = self.window()
        if not lo <= t <= hi:
            raise WindowError(f"time step {t} outside [{lo}, {hi}]")

    def records_at(self, t, games=None):
        self._check(t)
        rec = self.e.export() if t == self.t else self.rows[t]["records"]
        return rec if games is None else rec[np.asarray(games, dtype=np.int64)]

    def _engine_at(self, t, games):
        rec = self.records_at(t, games)
        cfg = self.e.cfg
        return OracleEngine.from_records(rec, cfg.seed, k_battleless=cfg.k_battleless,
                                         max_moves=cfg.max_moves, auto_reset=bool(cfg.auto_reset),
                                         two_square=bool(cfg.two_square), sampler=cfg.sampler,
                                         chasing=bool(cfg.chasing), acting_obs=bool(cfg.acting_obs))

    def mask_at(self, t, games=None):
        return self._engine_at(t, games).mask()

    def obs_at(self, t, games=None):
        return self._engine_at(t, games).encode()

    def info_at(self, t, games=None):
        """The App. B.1 scalar and per-square queries, from their definitions."""
        self._check(t)
        lo, _ = self.window()
        n_all = self.e.n
        ids = np.arange(n_all) if games is None else np.asarray(games, dtype=np.int64)
        rec = self.records_at(t)
        eng = self._engine_at(t, ids)
        m = len(ids)
        out = dict(acting_player=np.zeros(m, np.int8), played_action=np.full(m, -1, np.int16),
                   num_moves=np.zeros(m, np.int32), moves_since_attack=np.zeros(m, np.int32),
                   reward_pl0=np.zeros(m, np.int8), terminated_since=np.zeros(m, np.int32),
                   has_legal_movement=np.zeros(m, np.uint8), flag_captured=np.zeros(m, np.uint8),
                   two_square_applies=np.zeros(m, np.uint8), chase_applies=np.zeros(m, np.uint8),
                   is_unknown=np.zeros((m, 100), np.uint8), piece_onehot=np.zeros((m, 24, 100), np.uint8))
        row = self.rows.get(t) if t < self.t else None
        for k, g in enumerate(ids):
            r = rec[g]
            ply = _u32(r, _PLY)
            p = ply & 1
            done = r[_DONE] != 0
            out["acting_player"][k] = p
            out["num_moves"][k] = ply
            out["moves_since_attack"][k] = _u32(r, _BATTLELESS)
            if row is not None:
                out["played_action"][k] = row["actions"][g]
                ended = bool(row["done"][g]) and not done
                if ended:
                    out["reward_pl0"][k] = row["outcome"][g]
                    out["flag_captured"][k] = int(row["reason"][g] == _REASON_FLAG)
            if done:
                since, u = 1, t - 1
                while u >= lo and self.rows[u]["records"][g][_DONE]:
                    since += 1
                    u -= 1
                out["terminated_since"][k] = since
            out["has_legal_movement"][k] = int((not done) and eng.has_legal_move(k, p))
            out["two_square_applies"][k] = int(eng.two_square_applies(k))
            out["chase_applies"][k] = int(eng.chase_applies(k))
            for s in range(100):
                pid = int(r[_BOARD + s])   # int8 in the record: >= 128 means empty or lake
                if pid >= 128:
                    continue
                w0 = _u32(r, _PIECES + 16 * pid)
                ptype, revealed = w0 & 15, (w0 >> 5) & 1
                own = (pid >= 40) == (p == 1)
                f = s if p == 0 else 99 - s
                out["piece_onehot"][k, (0 if own else 12) + ptype, f] = 1
                out["is_unknown"][k, f] = int((not own) and not revealed)
        return out
