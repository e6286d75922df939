/*
 * stratego.h - C ABI of the MI355X batched Stratego engine (libstratego.so).
 *
 * The engine advances N independent games of Stratego in lockstep on one GPU:
 * legal-move masks, uniform random move sampling, move application with battle
 * resolution, terminal and draw detection with optional auto-reset, and the
 * 488-channel information-state encoding of both players.  It follows the
 * paper's simulator description (arXiv 2511.07312, App. B: a single object over
 * N parallel games, ApplyActions over a tensor of N actions, independent reset
 * of terminated games, reset to non-initial states for search, no allocation
 * after construction) and its statement of the game (App. A) and infostate
 * (App. C).
 *
 * Conventions shared by every call
 *   - Squares are 10*row + col, 0..99.  Red (player 0) starts in rows 0-3 and
 *     moves first; blue (player 1) starts in rows 6-9.  Lakes are the 2x2
 *     blocks rows 4-5 x cols 2-3 and 6-7.
 *   - An action is 100*from + to in absolute squares (0..9999); -1 = no-op.
 *   - Masks are packed bitsets: uint64 mask[N][157], bit a of game g is
 *     (mask[g][a >> 6] >> (a & 63)) & 1; bits 10000..10047 are zero.
 *   - Observations are uint8 obs[N][2][488][10][10]: game, observer (0 red,
 *     1 blue), channel, row, col, in the observer's frame (blue's view is the
 *     board rotated by 180 degrees); with acting_obs_only, obs[N][1][488][10][10]
 *     holds the acting player's view only.  Indicator channels hold 1; channels
 *     12-35 and 41-42 hold round(255*x) of a probability or fraction; channels
 *     456-487 hold 0x01 at a move's destination and 0xFF (int8 -1) at its
 *     source (App. C).
 *   - A game state is a canonical 1536-byte record, little-endian: u32 game
 *     id at 0, u32 episode at 4, i32 ply at 8, i32 battleless moves at 12, u8
 *     move-ring count at 16, u8 done at 17, i8 outcome at 18, u8 reason at 19,
 *     u32 redraws at 20; per player p the two-square state at 24 + 8p (u8
 *     piece id, u8 square count 0 or 2-4, u8 squares[4]); u8 chase length at
 *     40 and u8 chasing player at 41; i8 board[100] at 64 (piece id, -1
 *     empty, -2 lake); u8 ring[32][2] of (from, to) at 164, the move of ply t
 *     in slot t mod 32; at 256 + 16 id four u32 words per piece id (0-39 red,
 *     40-79 blue): type, alive, revealed, moved, death cause and square, the
 *     history-feature bits of App. C.1, and (word 0 bit 30) whether the piece
 *     ever moved more than one square, which App. A allows only a Scout, so
 *     that its type is public.  Records are the checkpoint format: importing
 *     an exported record continues the game bit-exactly.
 *   - Every device pointer must be device memory on the context's device.
 *     The caller owns all buffers it passes; the library owns the game states
 *     (allocated once in stratego_init).
 *   - Every call is asynchronous on the HIP stream given at init, except
 *     stratego_get_error, stratego_autotune, stratego_serve,
 *     stratego_board_strings and stratego_destroy, which synchronise it.
 *   - Return value: STRATEGO_OK (0) or a negative error code.  No C++
 *     exception crosses this interface.
 */
#ifndef STRATEGO_H
#define STRATEGO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STRATEGO_OK 0
#define STRATEGO_E_INVAL (-1)          /* bad argument (null pointer, size, range) */
#define STRATEGO_E_NOMEM (-2)          /* device allocation failed in stratego_init */
#define STRATEGO_E_HIP (-3)            /* a HIP runtime call failed */
#define STRATEGO_E_ILLEGAL_ACTION (-4) /* a live game received an illegal action */
#define STRATEGO_E_BAD_STATE (-5)      /* an imported record is malformed */
#define STRATEGO_E_RANGE (-6)          /* time step outside the rollout buffer's window */

#define STRATEGO_NUM_CHANNELS 488
#define STRATEGO_MASK_WORDS 157
#define STRATEGO_RECORD_BYTES 1536
#define STRATEGO_OBS_BYTES_PER_GAME 97600
#define STRATEGO_HISTORY_BYTES_PER_GAME_STEP 1544  /* rollout buffer: record + step outcome */
#define STRATEGO_MAX_LEGAL 256   /* legal-list capacity; a position has at most 244 legal moves */
#define STRATEGO_SAMPLER_UNIFORM 0
#define STRATEGO_SAMPLER_MAGNET 1

typedef struct stratego_ctx stratego_ctx;

typedef struct {
  int32_t num_games;      /* N, fixed for the life of the context */
  int32_t k_battleless;   /* draw after k consecutive battleless moves (App. D.1: 100) */
  int32_t max_moves;      /* draw at this many moves (App. D.1: 4000), >= 1 */
  int32_t auto_reset;     /* 1: a terminated game restarts with a fresh setup (App. B) */
  uint64_t seed;          /* Philox4x32-10 key for setups, moves and resampling */
  uint32_t game_id_base;  /* global game id of slot 0; slot i has id base + i */
  int32_t games_per_wg;   /* fused engine tile size G in {1,2,4,8,16}; 0 = default */
  int32_t lds_layout;     /* observation staging in LDS: 1 = bit planes of both players; 2..6 =
                             byte images in 1, 2, 4, 8, 16 channel segments; 7 = bit planes of
                             one player at a time (half the LDS); 0 = default (1) */
  int32_t history_len;    /* rollout buffer: time steps kept (App. B.1), 0..2^20; 0 = none */
  int32_t two_square_rule; /* 1: a piece may not cross the same square boundary on more than
                              three consecutive turns of its owner (App. A, App. B.2) */
  int32_t sampler;         /* move sampler of stratego_sample_actions and the fused plies:
                              0 uniform over legal actions; 1 magnet policy (section 2.4: a
                              piece with a legal move uniformly, then one of its moves) */
  int32_t chasing_rule;    /* 1: continuous-chasing rule (App. A, Table "chase", App. B.3): the
                              chasing player may not make a threat that recreates a position
                              of the chase (board and side to move, within the last 32 plies),
                              unless the moved piece returns to its square before that
                              player's previous turn */
  int32_t acting_obs_only; /* 1: every observation output holds only the acting player's
                              information state, uint8[N][1][488][10][10] (App. B.1
                              ComputeInfostateTensor); 0: both players, [N][2][488][10][10] */
} stratego_config;

/* Create a context with N games, all reset to fresh setups (episode 0).
 * hip_stream: a hipStream_t (NULL = the null stream).  Allocates every device
 * buffer the context will use.  Errors: E_INVAL, E_NOMEM, E_HIP. */
int stratego_init(const stratego_config* cfg, void* hip_stream, stratego_ctx** out);

/* Reset games (App. B: reset of terminated games; reset to a non-initial state
 * for search).  slots_dev: int32[n] slot indices, or NULL for slots 0..n-1.
 * states_dev: NULL = fresh uniform setups with episode 0 (a setup that is
 * already terminal is redrawn when auto_reset is on); otherwise n canonical
 * records copied into the slots.  A malformed record (lakes not exactly on
 * the lake squares, a board entry out of range or naming a dead piece, an
 * alive piece not on exactly one square, a player's types not the initial
 * multiset, a moved Flag or Bomb, a long-move bit on a piece that is not a
 * moved Scout, a dead piece unrevealed or with a bad death
 * cause or square, ring squares or counters out of range, malformed
 * two-square or chase state) or a slot outside [0, N) latches E_BAD_STATE in
 * the error word (see stratego_get_error) and leaves that slot unchanged. */
int stratego_reset(stratego_ctx* ctx, const int32_t* slots_dev, int32_t n, const void* states_dev);

/* Legal-action mask of the acting player of every game (App. B
 * ComputeLegalActionMask; App. A movement rules).  mask_dev: uint64[N][157].
 * num_legal_dev: int16[N] or NULL.  Finished games get an all-zero mask. */
int stratego_legal_mask(stratego_ctx* ctx, uint64_t* mask_dev, int16_t* num_legal_dev);

/* One uniformly random legal action per game (App. B SampleRandomLegalAction):
 * the r-th set bit of the mask in ascending action order, with
 * r = (u * n) >> 32, u = word x of Philox4x32-10(key = seed,
 * counter = (game id, ply, episode, 0)), n = num_legal.  -1 when n == 0. */
int stratego_sample_actions(stratego_ctx* ctx, const uint64_t* mask_dev,
                            const int16_t* num_legal_dev, int16_t* actions_dev);

/* Apply one action per game (App. B ApplyActions; App. A battles; App. C.1
 * history features).  actions_dev: int16[N]; -1 = no-op.  Outputs (each
 * int8/uint8/int16 [N], any may be NULL): done = 1 if the game is terminal
 * after this call (with auto-reset: it ended in this call and was restarted),
 * outcome (+1 red won, -1 blue won, 0 draw), reason (1 flag captured, 2 forced
 * win, 3 forced draw, 4 k-move rule, 5 maximum length), ep_len = moves in the
 * finished episode; all zero for games that are not done.  An illegal action
 * for a live game leaves that game unchanged and latches
 * E_ILLEGAL_ACTION with the lowest such slot. */
int stratego_step(stratego_ctx* ctx, const int16_t* actions_dev, int8_t* done_dev,
                  int8_t* outcome_dev, uint8_t* reason_dev, int16_t* ep_len_dev);

/* Information states of both players (App. C): obs_dev uint8[N][2][488][10][10]
 * (with acting_obs_only, uint8[N][1][488][10][10]: the acting player's).
 * Errors: E_INVAL (NULL obs_dev). */
int stratego_encode_obs(stratego_ctx* ctx, uint8_t* obs_dev);

/* Copy the N canonical records (1536 bytes each) to states_dev (device).  The
 * records are the compact state the paper's simulator keeps per game, from
 * which masks and information states are recomputed on demand (App. B, B.1);
 * imported with stratego_reset they restore the games exactly (a checkpoint,
 * or a snapshot of states for search). */
int stratego_export_states(stratego_ctx* ctx, void* states_dev);

/* Fused engine (one persistent kernel per ply): the step loop of the paper's
 * data collection and rollouts (App. B: the simulator advances all games in
 * lockstep; section 2.6, App. D.2: self-play generation), with the calls above
 * fused.  For each of nplies plies and
 * every game, legal mask -> sample (the context's sampler) -> encode the
 * observations of the pre-move state (both players, or the acting player's
 * with acting_obs_only) -> step (with the context's auto-reset).  The per-ply
 * outputs mask_dev, num_legal_dev and obs_dev are overwritten each ply (they
 * hold the last ply's values); actions/done/outcome/reason/ep_len are written
 * per ply as [nplies][N] arrays.  Any output may be NULL (obs_dev NULL skips
 * the encoding).  With use_graph = 1 the nplies launches are captured once
 * into a hipGraph (per distinct argument set) and replayed; use_graph = 2
 * only builds and uploads that graph (nothing runs, no game advances), so
 * that a later use_graph = 1 call with the same arguments starts at once.
 * ply_ns_dev, if
 * not NULL, receives int64[nplies] per-ply device durations in nanoseconds
 * (first wave start to last wave end).  Errors: E_INVAL (nplies < 0; use_graph
 * outside 0..2; nplies above 4096 with use_graph or ply_ns_dev), E_HIP. */
int stratego_run_plies(stratego_ctx* ctx, int32_t nplies, uint64_t* mask_dev,
                       int16_t* num_legal_dev, int16_t* actions_dev, uint8_t* obs_dev,
                       int8_t* done_dev, int8_t* outcome_dev, uint8_t* reason_dev,
                       int16_t* ep_len_dev, int32_t use_graph, int64_t* ply_ns_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc): stratego_run_plies
 * without a context or a graph, over caller-owned records.  states_dev:
 * uint8[cfg->num_games][1536] canonical records as the library writes them
 * (stratego_export_states, stratego_history_export, or an earlier call of
 * this function), advanced in place; slot i is game i.  cfg gives the rules,
 * the sampler, the observation mode and the tiling as for stratego_init
 * (num_games, k_battleless, max_moves, auto_reset, seed, two_square_rule,
 * sampler, chasing_rule, acting_obs_only, games_per_wg, lds_layout);
 * game_id_base is not used (records carry their game ids) and history_len
 * must be 0.  Outputs as for stratego_run_plies, any may be NULL.  The call
 * allocates nothing: the per-ply work counters of the persistent kernel sit
 * in a static device array of STRATEGO_STATIC_MAX_PLIES counters that each
 * device holds for the life of the process and that every call on that
 * device reuses (the first call on a device also looks up that array's
 * address and the device's limits).  Calls that overlap on one device
 * (different streams, or different host threads without ordering) race on
 * the counters and must not be made.  Asynchronous on hip_stream (NULL = the
 * null stream), which must belong to the current device.  Drawn actions are
 * legal by construction, so no error word is kept.  Errors: E_INVAL (NULL
 * cfg or states_dev, an invalid cfg field, nplies outside [0,
 * STRATEGO_STATIC_MAX_PLIES], more devices than the library tracks), E_HIP. */
#define STRATEGO_STATIC_MAX_PLIES 4096
int stratego_run_plies_static(const stratego_config* cfg, void* hip_stream, void* states_dev, int32_t nplies,
                              uint64_t* mask_dev, int16_t* num_legal_dev, int16_t* actions_dev,
                              uint8_t* obs_dev, int8_t* done_dev, int8_t* outcome_dev, uint8_t* reason_dev,
                              int16_t* ep_len_dev);

/* Same as stratego_run_plies over a subset of slots (serving): slots_dev
 * int32[nslots] (distinct, each in [0, N); an out-of-range entry is skipped
 * and latches E_BAD_STATE with its list position); per-game outputs are
 * indexed by position in the slot list ([nplies][nslots], obs
 * [nslots][2 or 1][488][100]).  No graph.  Errors: E_INVAL (NULL slots_dev,
 * nslots outside [0, N], nplies < 0, a rollout buffer present), E_HIP. */
int stratego_run_plies_slots(stratego_ctx* ctx, const int32_t* slots_dev, int32_t nslots,
                             int32_t nplies, uint64_t* mask_dev, int16_t* actions_dev,
                             uint8_t* obs_dev, int8_t* done_dev, int8_t* outcome_dev,
                             uint8_t* reason_dev, int16_t* ep_len_dev);

/* Search support (paper section 2.5, App. B reset to non-initial states):
 * slot i*per + j (i < nsrc, j < per) receives src record i with the hidden
 * types of the player not to move redrawn uniformly among assignments
 * consistent with public information (revealed and dead pieces keep their
 * types; a piece that has moved is neither Flag nor Bomb), drawn from
 * Philox4x32-10(key = seed, counter = (new id, block, episode, 3)); the new
 * game id is game_id_base + i*per + j; a piece seen moving more than one
 * square keeps its type (a known Scout); slots from nsrc*per on are left as
 * they are.  A malformed source record latches E_BAD_STATE with the slot of
 * its first resample (i*per) and its slots are left as they are.  Errors:
 * E_INVAL (null source, nsrc or per below 1, nsrc*per above N, a device with
 * less than 80 KB of LDS per workgroup), E_HIP. */
int stratego_reset_resampled(stratego_ctx* ctx, const void* src_states_dev, int32_t nsrc,
                             int32_t per, uint32_t game_id_base);

/* Serving (continuous batching).  A request asks for `plies` fused plies of
 * num_games games whose canonical records sit at rows [first, first +
 * num_games) of in_states_dev.  Kinds: STRATEGO_REQ_STEP (plies must be 1; the
 * observations of the input states (both players, or the acting player's with
 * acting_obs_only) are written to obs_out_dev
 * at rows first + j, or at the game's pool slot when obs_by_slot = 1) and
 * STRATEGO_REQ_ROLLOUT (no observations).  The context's N slots are the
 * device-resident pool.  Requests are admitted in arrival order, once they
 * have arrived (realtime = 1: at arrival_s seconds after the call starts;
 * realtime = 0: all at once) and while both enough free slots and enough of
 * the memory budget remain (a game reserves 1536 bytes, plus its observation
 * bytes, 97600 or 48800, for step requests); mem_budget_bytes <= 0 uses the
 * device's free memory at the start of the call.  A request that does not
 * fit lets later arrived requests that fit go ahead of it (backfilling) until
 * it has waited backfill_wait_s seconds since its arrival (since the call's
 * start with realtime = 0); from then on nothing is admitted before it, so it
 * enters as soon as enough slots have freed.  backfill_wait_s < 0 admits in
 * strict arrival order.  Every iteration runs one
 * fused ply over all admitted games, so requests that arrive while others run
 * join them on the device; a request leaves after its last ply, when its
 * final records are copied to rows [first, first + num_games) of
 * out_states_dev.  The host enqueues an iteration while the previous one runs
 * (two in flight), and imports admitted records on a second stream of the
 * context beside them; a request's slots are reused once the iteration that
 * copied it out has completed.  results[r] receives the host time of
 * admission and the time the device completed the request's last iteration
 * (device event time placed on the host clock).  Each game's result depends
 * only on its record, so it is the same alone and in any mix.  The error word
 * latches E_BAD_STATE for a malformed input record (that game then runs from
 * whatever its slot held).  Synchronises the stream.  Errors: E_INVAL (bad
 * request, a request that can never fit, step requests without obs_out_dev,
 * a NaN backfill_wait_s), E_HIP. */
#define STRATEGO_REQ_STEP 0
#define STRATEGO_REQ_ROLLOUT 1
typedef struct {
  int32_t kind;
  int32_t plies;
  int32_t num_games;
  int32_t first;
  double arrival_s;
} stratego_request;
typedef struct {
  double admit_s;
  double done_s;
} stratego_request_result;
typedef struct {
  double wall_s;                /* host time of the whole call */
  int64_t game_steps;
  int32_t iterations;
  int32_t peak_active_games;
  int64_t peak_reserved_bytes;
  int64_t budget_bytes;
  double gpu_busy_s;            /* device time inside iterations (their plies and copies out) */
  double gpu_span_s;            /* device time from the first iteration's start to the last one's end;
                                   1 - busy / span is the share the device idled between iterations */
} stratego_serve_stats;
int stratego_serve(stratego_ctx* ctx, const stratego_request* reqs, int32_t nreq,
                   const void* in_states_dev, void* out_states_dev, uint8_t* obs_out_dev,
                   int32_t obs_by_slot, int64_t mem_budget_bytes, int32_t realtime,
                   double backfill_wait_s, stratego_request_result* results,
                   stratego_serve_stats* stats);

/* Time the fused engine for every (games_per_wg, lds_layout) pair that fits
 * the device, plies plies each, restoring the game states afterwards, and
 * adopt the fastest.  report (may be NULL) receives up to max_entries rows of
 * {games_per_wg, lds_layout, microseconds per ply}; returns the number of
 * rows through n_entries.  Synchronises the stream. */
typedef struct {
  int32_t games_per_wg;
  int32_t lds_layout;
  double us_per_ply;
} stratego_tune_entry;
int stratego_autotune(stratego_ctx* ctx, uint8_t* obs_dev, uint64_t* mask_dev, int32_t plies,
                      stratego_tune_entry* report, int32_t max_entries, int32_t* n_entries);

/* Current fused-engine tiling (games per workgroup, LDS layout). */
int stratego_get_tiling(stratego_ctx* ctx, int32_t* games_per_wg, int32_t* lds_layout);
int stratego_set_tiling(stratego_ctx* ctx, int32_t games_per_wg, int32_t lds_layout);

/* Rollout buffer (App. B.1: the simulator doubles as the rollout buffer; past
 * legal masks and information states are recomputed on demand from a
 * circular, preallocated history instead of being stored).
 *
 * Time steps count whole-batch plies: t = 0 is the state after init, and each
 * stratego_step or fused ply of stratego_run_plies maps the states at t to
 * those at t + 1.  With history_len = H > 0, every such ply records, for each
 * game, the state the action is applied to (its canonical record) and the
 * step's outcome, in ring row t mod H; stratego_init allocates H x N x 1544
 * bytes for this (against 98,856 bytes per game step for storing the mask and
 * both information states instead).  Queries accept
 * t in [max(0, T - H), T], T being the current time step, and return E_RANGE
 * otherwise; t = T reads the live states (resets and imports made since the
 * last ply included).  With H > 0, stratego_run_plies_slots and
 * stratego_serve, which step subsets of the games, return E_INVAL.
 *
 * Every query takes games_dev: int32[count] game indices (duplicates
 * allowed), or NULL for games 0..count-1 (count <= N); outputs are indexed by
 * position in that list.  An index outside [0, N) is skipped and latches
 * E_BAD_STATE with its list position (stratego_get_error).  count = 0 is a
 * no-op (outputs may then be NULL).  Queries are asynchronous on the
 * context's stream. */

/* The query window: *oldest = max(0, T - H), *current = T (either may be NULL). */
int stratego_history_window(stratego_ctx* ctx, int64_t* oldest, int64_t* current);

/* ComputeLegalActionMask(t) of App. B.1: mask_dev uint64[count][157] and/or
 * num_legal_dev int16[count] (either may be NULL, not both), as
 * stratego_legal_mask would have returned at time step t. */
int stratego_history_legal_mask(stratego_ctx* ctx, int64_t t, const int32_t* games_dev, int32_t count,
                                uint64_t* mask_dev, int16_t* num_legal_dev);

/* ComputeInfostateTensor(t) of App. B.1: obs_dev uint8[count][2][488][10][10],
 * both players' information states (App. C) at time step t, as
 * stratego_encode_obs would have returned then (uint8[count][1][488][10][10],
 * the acting player's, with acting_obs_only). */
int stratego_history_encode_obs(stratego_ctx* ctx, int64_t t, const int32_t* games_dev, int32_t count,
                                uint8_t* obs_dev);

/* Scalar and per-square queries of App. B.1 at time step t.  Every pointer is a
 * device array indexed by list position and may be NULL.  "The action at t"
 * is the one applied to the state at t (none yet at t = T).
 *   acting_player       int8:  0 red, 1 blue (ActingPlayer)
 *   played_action       int16: the action at t, -1 at t = T (GetPlayedActions)
 *   num_moves           int32: moves played in the episode (GetNumMoves)
 *   moves_since_attack  int32: consecutive moves without a battle
 *                              (GetNumMovesSinceLastAttack)
 *   reward_pl0          int8:  outcome for red (+1, 0, -1) if the action at t
 *                              ended the episode, else 0 (ComputeRewardPl0)
 *   terminated_since    int32: 0 for a live game; for a finished one, the
 *                              number of consecutive terminal states up to t in
 *                              the window (GetTerminatedSince; only games
 *                              without auto-reset stay finished)
 *   has_legal_movement  uint8: the acting player has a legal move in a live
 *                              game (GetHasLegalMovement)
 *   flag_captured       uint8: the action at t captured a Flag (GetFlagCaptured)
 *   two_square_applies  uint8: the two-square rule is on and removes at least
 *                              one move the acting player could otherwise make
 *                              (ComputeTwoSquareRuleApplies)
 *   chase_applies       uint8: the chasing rule is on and removes at least one
 *                              move the acting player could otherwise make
 *   is_unknown          uint8 [count][100]: 1 on squares holding an opponent
 *                              piece whose type the acting player has not seen
 *                              (ComputeIsUnknownPiece), acting player's frame
 *   piece_onehot        uint8 [count][24][100]: plane k < 12 marks the acting
 *                              player's pieces of type k, plane 12 + k the
 *                              opponent's (true types; ComputePieceTypeOnehot),
 *                              acting player's frame */
typedef struct {
  int8_t* acting_player;
  int16_t* played_action;
  int32_t* num_moves;
  int32_t* moves_since_attack;
  int8_t* reward_pl0;
  int32_t* terminated_since;
  uint8_t* has_legal_movement;
  uint8_t* flag_captured;
  uint8_t* is_unknown;
  uint8_t* piece_onehot;
  uint8_t* two_square_applies;
  uint8_t* chase_applies;
} stratego_history_outputs;
int stratego_history_info(stratego_ctx* ctx, int64_t t, const int32_t* games_dev, int32_t count,
                          const stratego_history_outputs* out);

/* Canonical records (1536 bytes each) of the listed games at time step t, to
 * states_dev uint8[count][1536]: importing them with stratego_reset rewinds
 * those games to t (App. B.1: capturing past states for search). */
int stratego_history_export(stratego_ctx* ctx, int64_t t, const int32_t* games_dev, int32_t count,
                            void* states_dev);

/* BoardStrs of App. B (a debugging aid): a picture of each listed game's
 * board at time step t (any step of the rollout buffer's window, as for the
 * queries above).  Rows 9 down to 0, one text line each; per square three
 * characters: the owner ('r' red, 'b' blue) and the type symbol (S Spy, 2
 * Scout, 3 Miner, 4-9 Sergeant to General, M Marshal, F Flag, B Bomb), "~~"
 * for a lake or ".." for an empty square, then a space (a newline after
 * column 9).  out_host: host memory, count slots of
 * STRATEGO_BOARD_STRING_BYTES bytes, each a NUL-terminated string.
 * games_dev: int32[count] game indices (device memory) or NULL for games
 * 0..count-1.  Synchronises the stream.  Errors: E_INVAL (an index outside
 * [0, N), NULL out_host), E_RANGE, E_HIP. */
#define STRATEGO_BOARD_STRING_BYTES 301
int stratego_board_strings(stratego_ctx* ctx, int64_t t, const int32_t* games_dev, int32_t count,
                           char* out_host);

/* Policies over legal lists (sections 2.4-2.5 and App. D.7).  A game's legal list
 * is its acting player's legal actions in ascending order, padded to
 * STRATEGO_MAX_LEGAL entries with -1 (finished games: all -1).  Per-action
 * arrays are float[N][256] aligned with the list; entries past num_legal are
 * ignored on input and written as 0 on output. */

/* actions_dev int16[N][256]: the legal lists; num_legal_dev int16[N] or NULL. */
int stratego_legal_list(stratego_ctx* ctx, int16_t* actions_dev, int16_t* num_legal_dev);

/* The magnet policy rho (section 2.4 / App. D.4: a piece with a legal move
 * uniformly at random, then one of its legal moves uniformly at random):
 * probs_dev float[N][256], rho = 1 / (P * m) as one IEEE single division,
 * P = pieces with a legal move, m = legal moves of the listed action's piece. */
int stratego_magnet_policy(stratego_ctx* ctx, float* probs_dev);

/* The search policy of App. D.7: the maximiser of <q, pi> - alpha KL(pi, rho)
 * - beta KL(pi, pi_theta), i.e. pi proportional to [exp(q) rho^alpha
 * pi_theta^beta]^(1 / (alpha + beta)), over each legal list, in single
 * precision.  q_dev: advantage estimates, logpi_dev: log pi_theta, both
 * float[N][256]; alpha, beta >= 0 with alpha + beta > 0 (the paper's search
 * uses alpha = 0.002, beta = 0.02).  probs_dev float[N][256]. */
int stratego_search_policy(stratego_ctx* ctx, const float* q_dev, const float* logpi_dev, float alpha,
                           float beta, float* probs_dev);

/* One action per game from a distribution over its legal list (probs_dev
 * float[N][256]): u = the top 24 bits of word x of Philox4x32-10(key = seed,
 * counter = (game id, ply, episode, 4)) as a fraction; the first listed
 * action whose single-precision running sum, in list order, exceeds u times
 * the single-precision total; the last action with a positive weight if
 * rounding leaves none; -1 for an empty list.  actions_dev int16[N]. */
int stratego_sample_policy(stratego_ctx* ctx, const float* probs_dev, int16_t* actions_dev);

/* Synchronise the stream, then report and clear the latched device error:
 * returns STRATEGO_OK, E_ILLEGAL_ACTION or E_BAD_STATE; first_bad_slot (may
 * be NULL) receives the lowest offending slot or -1. */
int stratego_get_error(stratego_ctx* ctx, int32_t* first_bad_slot);

/* Number of state updates (game steps) applied by step/run_plies so far
 * (App. B CurrentStep). */
int stratego_current_step(stratego_ctx* ctx, int64_t* steps);

/* Synchronise and free everything the context owns. */
int stratego_destroy(stratego_ctx* ctx);

/* Static description of an error code. */
const char* stratego_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* STRATEGO_H */
