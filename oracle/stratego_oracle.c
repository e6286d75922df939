/*
 * Stratego rules oracle: a plain, slow, scalar CPU implementation of the
 * batched game engine's semantics (setup, legal moves, uniform move
 * sampling, move application with battles and history features, terminal
 * and draw detection, auto-reset, the 488-channel information-state
 * encoding, and the search-shaped hidden-type resampler).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU engine.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or constant generator with the
 * HIP engine; both sides are written independently from the paper and from
 * the written readings of it.
 *
 * Paper references are to arXiv 2511.07312 ("Superhuman AI for Stratego"):
 *   App. A  (Rules of Stratego, incl. Table "pieces")
 *   App. B  (GPU simulator: reset behaviour, API table, auto-reset)
 *   App. C  (Information state: C.1 board channels 0-455, C.2 recent moves)
 *   App. D.1 (game-rule hyper-parameters: k-move rule, max game length)
 *   App. B.2 (two-square rule state machine)
 *   App. B.3 (continuous-chasing rule)
 *
 * Pinning status of each part (how the tests tie it to something other
 * than itself):
 *   battle outcome ............ pinned: full 10x12 table fixture from Table pieces
 *   legal moves ............... pinned: brute-force pairwise predicate, closed form at ply 0
 *   setup shuffle ............. pinned: multiset/row invariants, uniformity test, and the
 *                               Durstenfeld convention recomputed for 1000 game ids
 *   Philox4x32-10 ............. pinned: SC'11 known-answer vectors + an independent library
 *   move samplers ............. pinned: the uniform (word x) and magnet (words y, z)
 *                               conventions recomputed for 1000 games x 24 plies
 *   terminal logic ............ pinned: hand-built positions for every reason
 *   probability channels ...... pinned: brute-force enumeration of consistent assignments
 *                               (known Scouts included), hand-built closed forms
 *   history features .......... pinned against the readings of App. C.1's words
 *                               (the paper prints no worked example): a brute
 *                               force recomputes every ply's increments from the
 *                               boards before and after the move in whole random
 *                               games, plus hand-built scenarios
 *   encoding layout ........... pinned: every channel group against planes written
 *                               by hand from the App. C.1 / C.2 tables (both frames,
 *                               move planes most recent first), plus invariants
 *   resampler ................. pinned by invariants, by agreement of its empirical
 *                               frequencies with the probability channels, and by
 *                               its convention recomputed for 1024 resamples
 *   two-square rule ........... pinned by hand-built move sequences written
 *                               from the rule's statement (App. A), including
 *                               Scout spans (the Scout case is a reading), and by
 *                               a brute force that rebuilds each player's run
 *                               from the move record in random games
 *   chasing rule .............. pinned by hand-built chases written from the
 *                               rule's statement and Table "chase", and by a
 *                               brute force that undoes the whole board
 *                               history in chase-driven games; threat, evasion
 *                               and the position window are readings
 *   acting-player encoding .... pinned: equals the acting observer's half of
 *                               the both-player encoding
 *   magnet policy ............. pinned by closed forms (a lone Scout, two
 *                               pieces) and by sampled piece and move
 *                               frequencies (section 2.4, App. D.4)
 *   search policy ............. pinned by optimality: it beats random points of
 *                               the simplex on the regularised objective, and
 *                               reduces to rho when q = 0 and pi_theta = rho
 *                               (App. D.7)
 *   policy sampler ............ pinned by sampled frequencies and by never
 *                               drawing a zero-weight action
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <math.h>

/* ------------------------------------------------------------------ */
/* Pieces (App. A, Table "pieces").  Type index follows the channel order
 * of App. C.1 channels 0-11: Spy, Scout, Miner, Sergeant, Lieutenant,
 * Captain, Major, Colonel, General, Marshal, Flag, Bomb.                */
enum { SPY = 0, SCOUT, MINER, SERGEANT, LIEUTENANT, CAPTAIN, MAJOR, COLONEL,
       GENERAL, MARSHAL, FLAG, BOMB, NUM_TYPES };

static const int INITIAL_COUNT[NUM_TYPES] = {1, 8, 5, 4, 4, 4, 3, 2, 1, 1, 1, 6};

#define NSQ 100
#define NPIECES 80
#define NCHAN 488
#define PLANE 100
#define MASK_WORDS 157
#define RING 32
#define EMPTY (-1)
#define LAKE (-2)

enum { REASON_NONE = 0, REASON_FLAG = 1, REASON_FORCED_WIN = 2,
       REASON_FORCED_DRAW = 3, REASON_KMOVE = 4, REASON_MAXMOVES = 5 };

enum { BATTLE_ATTACKER = 0, BATTLE_DEFENDER = 1, BATTLE_TIE = 2 };

enum { TAG_MOVE = 0, TAG_SETUP0 = 1, TAG_SETUP1 = 2, TAG_RESAMPLE = 3, TAG_POLICY = 4 };
enum { SAMPLER_UNIFORM = 0, SAMPLER_MAGNET = 1 };

typedef struct {
    uint64_t seed;
    int32_t k_battleless;   /* k of the k-move rule (App. D.1: 100 in training) */
    int32_t max_moves;      /* maximum game length (App. D.1: 4000) */
    int32_t auto_reset;     /* reset terminated games to a fresh setup (App. B) */
    int32_t two_square;     /* enforce the two-square rule (App. A competitive play) */
    int32_t sampler;        /* move sampler: 0 uniform over legal actions, 1 magnet policy */
    int32_t chasing;        /* enforce the continuous-chasing rule (App. A competitive play) */
    int32_t acting_obs;     /* encode only the acting player's information state (App. B.1) */
    int32_t pad;
} orc_cfg;

/* rule flags passed to the move generator */
enum { RULE_TWO_SQUARE = 1, RULE_CHASING = 2 };
static int rules_of(const orc_cfg* cfg) {
    return (cfg->two_square ? RULE_TWO_SQUARE : 0) | (cfg->chasing ? RULE_CHASING : 0);
}

typedef struct {
    int type;
    int alive;
    int revealed;
    int moved;
    int long_move;      /* once moved more than one square in one move (only a Scout can) */
    int death_square;   /* -1 while alive */
    int death_cause;    /* 0 while alive, else 1..6 (App. C.1 "Causes of death") */
    /* "has ever" sets (App. C.1): 11-bit sets, bit i < 10 = revealed type i,
     * bit 10 = hidden */
    unsigned threat, evade, adj;
    /* 13-bit protection sets: bits 0..10 = revealed type (Spy..Marshal, Bomb),
     * bit 11 = empty square (only for prot) / padding, bit 12 = hidden */
    unsigned prot, prot_against, been_by, been_against;
} orc_piece;

typedef struct {
    uint32_t game_id;
    uint32_t episode;
    int ply;            /* moves made in this episode; red acts when even */
    int battleless;     /* consecutive moves without a battle */
    int board[NSQ];     /* piece id, EMPTY or LAKE */
    orc_piece piece[NPIECES];
    int ring_count;
    int ring_from[RING];
    int ring_to[RING];
    int done;
    int outcome;
    int reason;
    uint32_t redraws;
    /* two-square rule state of each player (App. B.2): the piece that player
     * moved last and the squares it occupied, oldest first, ending on its
     * current square (ts_n = 0: none; at most 4, i.e. three moves) */
    int ts_piece[2];
    int ts_n[2];
    int ts_pos[2][4];
    /* continuous-chasing state (App. A Table "chase"): the number of plies of
     * the current chase (alternating threats by `chaser` and evasions by the
     * other side, 0 = none, at most 255) and the chasing player */
    int chase_len;
    int chaser;
} orc_state;

/* ------------------------------------------------------------------ */
/* Board geometry (App. A: 10x10, 92 occupiable squares, two 2x2 lakes in
 * the middle rows).  Square index = 10*row + col.                       */
static int is_lake(int sq) {
    int r = sq / 10, c = sq % 10;
    return (r == 4 || r == 5) && (c == 2 || c == 3 || c == 6 || c == 7);
}

static int owner_of(int id) { return id < 40 ? 0 : 1; }

/* Start square implied by the piece id: red id i starts on square i, blue
 * id 40+i starts on square 99-i. */
static int start_square(int id) { return id < 40 ? id : 99 - (id - 40); }

static int is_movable_type(int t) { return t != FLAG && t != BOMB; }

/* On-board orthogonal neighbours, written to nb[]; returns their count. */
static int neighbours(int sq, int nb[4]) {
    int r = sq / 10, c = sq % 10, n = 0;
    if (r > 0) nb[n++] = sq - 10;
    if (r < 9) nb[n++] = sq + 10;
    if (c > 0) nb[n++] = sq - 1;
    if (c < 9) nb[n++] = sq + 1;
    return n;
}

static int adjacent(int a, int b) {
    int ra = a / 10, ca = a % 10, rb = b / 10, cb = b % 10;
    int dr = ra - rb, dc = ca - cb;
    if (dr < 0) dr = -dr;
    if (dc < 0) dc = -dc;
    return dr + dc == 1;
}

/* ------------------------------------------------------------------ */
/* Battle outcome (App. A, Table pieces).  Attacker type a is movable.    */
int orc_battle(int a, int d) {
    if (d == FLAG) return BATTLE_ATTACKER;                 /* Flag loses to any attacker */
    if (d == BOMB) return a == MINER ? BATTLE_ATTACKER     /* Miner defeats Bomb */
                                     : BATTLE_DEFENDER;    /* Bomb defeats other attackers */
    if (a == SPY && d == MARSHAL) return BATTLE_ATTACKER;  /* Spy defeats Marshal when attacking */
    /* otherwise by rank: rank = type index + 1 for Spy..Marshal */
    if (a > d) return BATTLE_ATTACKER;
    if (a < d) return BATTLE_DEFENDER;
    return BATTLE_TIE;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random
 * numbers: as easy as 1, 2, 3").  Ten rounds of the 4x32 Philox S-box with
 * a Weyl-sequence key schedule.                                          */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof(c));
}

static void philox_block(uint64_t seed, uint32_t game_id, uint32_t a, uint32_t episode,
                         uint32_t tag, uint32_t out[4]) {
    uint32_t ctr[4] = {game_id, a, episode, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Uniform integer in [0, n) from one 32-bit word by multiply-shift. */
static uint32_t bounded(uint32_t u, uint32_t n) {
    return (uint32_t)(((uint64_t)u * (uint64_t)n) >> 32);
}

/* Sequential stream of 32-bit words: block j of a counter supplies words
 * x, y, z, w in that order. */
typedef struct {
    uint64_t seed;
    uint32_t game_id, episode, tag;
    uint32_t block;
    uint32_t words[4];
    int used;
} word_stream;

static void stream_init(word_stream* s, uint64_t seed, uint32_t game_id, uint32_t episode,
                        uint32_t tag) {
    s->seed = seed;
    s->game_id = game_id;
    s->episode = episode;
    s->tag = tag;
    s->block = 0;
    s->used = 4;
}

static uint32_t stream_next(word_stream* s) {
    if (s->used == 4) {
        philox_block(s->seed, s->game_id, s->block, s->episode, s->tag, s->words);
        s->block++;
        s->used = 0;
    }
    return s->words[s->used++];
}

/* ------------------------------------------------------------------ */
/* Legal moves (App. A "Piece details").  legal[100*from+to] = 1.         */
/* ------------------------------------------------------------------ */
/* Two-square rule (App. A: a piece may not cross the same square boundary
 * on more than three consecutive turns of its owner; App. B.2: tracked as
 * the last four squares of each player's last-moved piece).  A move from u
 * to v along a row or column crosses the unit boundaries between
 * consecutive squares of the segment; boundary k of a line lies between
 * coordinates k and k+1 of that line. */
typedef struct { int axis, line, lo, hi; } span;   /* boundaries lo..hi-1 */

static span move_span(int u, int v) {
    span sp;
    int ru = u / 10, cu = u % 10, rv = v / 10, cv = v % 10;
    if (ru == rv) { sp.axis = 0; sp.line = ru; sp.lo = cu < cv ? cu : cv; sp.hi = cu < cv ? cv : cu; }
    else          { sp.axis = 1; sp.line = cu; sp.lo = ru < rv ? ru : rv; sp.hi = ru < rv ? rv : ru; }
    return sp;
}

/* Would moving the player's piece from `from` to `to` cross, for the fourth
 * consecutive own turn, a boundary its last three moves all crossed? */
static int two_square_forbids(const orc_state* st, int player, int from, int to) {
    if (st->ts_n[player] < 4) return 0;
    const int* pos = st->ts_pos[player];
    if (pos[3] != from || st->board[from] != st->ts_piece[player]) return 0;
    span m[4] = {move_span(pos[0], pos[1]), move_span(pos[1], pos[2]), move_span(pos[2], pos[3]),
                 move_span(from, to)};
    int lo = m[0].lo, hi = m[0].hi;
    for (int i = 1; i < 4; i++) {
        if (m[i].axis != m[0].axis || m[i].line != m[0].line) return 0;
        if (m[i].lo > lo) lo = m[i].lo;
        if (m[i].hi < hi) hi = m[i].hi;
    }
    return lo < hi;
}

/* After the player's piece X moved from `from` to `to`: extend its record
 * when it is the same piece continuing from where it stopped, else start a
 * new one; forget it when the piece did not end on `to` (it died). */
static void two_square_update(orc_state* st, int player, int X, int from, int to) {
    if (st->board[to] != X) { st->ts_n[player] = 0; return; }
    int n = st->ts_n[player];
    int* pos = st->ts_pos[player];
    if (n > 0 && st->ts_piece[player] == X && pos[n - 1] == from) {
        if (n == 4) { pos[0] = pos[1]; pos[1] = pos[2]; pos[2] = pos[3]; n = 3; }
        pos[n++] = to;
    } else {
        st->ts_piece[player] = X;
        pos[0] = from;
        pos[1] = to;
        n = 2;
    }
    st->ts_n[player] = n;
}

static int chase_forbids(const orc_state* st, int player, int from, int to);

/* ------------------------------------------------------------------ */
/* Continuous-chasing rule (App. A and Table "chase"): a threat moves a piece
 * next to an enemy piece; an evasion moves a piece that the previous move
 * threatened away from its threatener; a chase is an unbroken alternation of
 * threats by one player and evasions by the other.  The chasing player may
 * not make a threat that recreates a position of the chase, unless the moved
 * piece returns to the square it held before that player's previous turn.
 * A position is the board together with the side to move, so the position a
 * threat creates (the opponent to move) can only equal one an odd number of
 * plies back.  The positions of the chase are rebuilt here by undoing the
 * moves of the move record on a copy of the board; the record keeps the
 * last 32 plies, so a chase is compared over at most that window. */
#define CHASE_WINDOW RING
static int threatens_after(const int board[NSQ], int sq, int player) {
    int nb[4], nn = neighbours(sq, nb);
    for (int i = 0; i < nn; i++) {
        int o = board[nb[i]];
        if (o >= 0 && owner_of(o) != player) return 1;
    }
    return 0;
}

static int chase_forbids(const orc_state* st, int player, int from, int to) {
    int L = st->chase_len;
    if (L < 2 || (L & 1) || st->chaser != player) return 0;   /* not the chaser's turn in a chase */
    if (st->board[to] != EMPTY) return 0;                      /* an attack is not a threat */
    int after[NSQ];
    memcpy(after, st->board, sizeof(after));
    after[to] = after[from];
    after[from] = EMPTY;
    if (!threatens_after(after, to, player)) return 0;
    int prev = (st->ply - 2) & (RING - 1);                     /* the chaser's previous move */
    if (st->ring_to[prev] == from && st->ring_from[prev] == to) return 0;
    int b[NSQ];
    memcpy(b, st->board, sizeof(b));
    int K = L < st->ring_count ? L : st->ring_count;           /* ring_count <= CHASE_WINDOW */
    for (int k = 1; k <= K; k++) {                             /* positions P_{L-1}, ..., P_{L-K} */
        int slot = (st->ply - k) & (RING - 1);
        int f = st->ring_from[slot], g = st->ring_to[slot];
        b[f] = b[g];
        b[g] = EMPTY;
        if ((k & 1) && memcmp(b, after, sizeof(b)) == 0) return 1;   /* same side to move */
    }
    return 0;
}

/* After player p's move from -> to (battle or not, with the previous move's
 * mover A on a, A = -1 if none): extend, restart or end the chase. */
static void chase_update(orc_state* st, int p, int battle, int from, int to, int A, int a) {
    int threat = !battle && threatens_after(st->board, to, p);
    int evade = !battle && A >= 0 && adjacent(from, a) && !adjacent(to, a);
    int L = st->chase_len;
    if (!battle && L > 0 && p == st->chaser && threat && !(L & 1)) L++;
    else if (!battle && L > 0 && p != st->chaser && evade && (L & 1)) L++;
    else if (threat) { L = 1; st->chaser = p; }
    else L = 0;
    if (L > 255) L = 255;
    st->chase_len = L;
    if (L == 0) st->chaser = 0;
}

static int legal_actions(const orc_state* st, int player, int rules, unsigned char* legal) {
    static const int DR[4] = {-1, 1, 0, 0};
    static const int DC[4] = {0, 0, -1, 1};
    int n = 0;
    if (legal) memset(legal, 0, 10000);
    for (int x = 0; x < NSQ; x++) {
        int id = st->board[x];
        if (id < 0 || owner_of(id) != player) continue;
        int t = st->piece[id].type;
        if (!is_movable_type(t)) continue;
        int maxk = (t == SCOUT) ? 9 : 1;
        for (int d = 0; d < 4; d++) {
            int r = x / 10, c = x % 10;
            for (int k = 1; k <= maxk; k++) {
                int rr = r + DR[d] * k, cc = c + DC[d] * k;
                if (rr < 0 || rr > 9 || cc < 0 || cc > 9) break;
                int y = rr * 10 + cc;
                if (is_lake(y)) break;
                int o = st->board[y];
                if (o >= 0 && owner_of(o) == player) break;
                if (!((rules & RULE_TWO_SQUARE) && two_square_forbids(st, player, x, y)) &&
                    !((rules & RULE_CHASING) && chase_forbids(st, player, x, y))) {
                    if (legal) legal[100 * x + y] = 1;
                    n++;
                }
                if (o != EMPTY) break;
            }
        }
    }
    return n;
}

/* A player has a legal move iff its legal list is not empty (with the
 * two-square rule on, the list already leaves out the forbidden moves). */
static int has_legal_move(const orc_state* st, int player, int rules) {
    return legal_actions(st, player, rules, NULL) > 0;
}

/* ------------------------------------------------------------------ */
/* Terminal check (App. A game summary, App. D.1 rule parameters).  The
 * priority order is a reading: flag capture, then no legal moves, then the
 * k-move rule, then the maximum length. */
static void terminal_check(orc_state* st, const orc_cfg* cfg, int flag_captured_by) {
    int q = st->ply & 1;
    if (flag_captured_by >= 0) {
        st->done = 1;
        st->outcome = flag_captured_by == 0 ? 1 : -1;
        st->reason = REASON_FLAG;
        return;
    }
    if (!has_legal_move(st, q, rules_of(cfg))) {
        st->done = 1;
        if (!has_legal_move(st, 1 - q, rules_of(cfg))) {
            st->outcome = 0;
            st->reason = REASON_FORCED_DRAW;
        } else {
            st->outcome = (1 - q) == 0 ? 1 : -1;
            st->reason = REASON_FORCED_WIN;
        }
        return;
    }
    if (st->battleless >= cfg->k_battleless) {
        st->done = 1;
        st->outcome = 0;
        st->reason = REASON_KMOVE;
        return;
    }
    if (st->ply >= cfg->max_moves) {
        st->done = 1;
        st->outcome = 0;
        st->reason = REASON_MAXMOVES;
        return;
    }
    st->done = 0;
    st->outcome = 0;
    st->reason = REASON_NONE;
}

/* ------------------------------------------------------------------ */
/* Setup: each player's 40 pieces uniformly at random in its own four back
 * rows (App. A), drawn by a Durstenfeld shuffle of the type multiset. */
static void shuffle_setup(uint64_t seed, uint32_t game_id, uint32_t episode, int player,
                          int types_out[40]) {
    int a[40], n = 0;
    for (int t = 0; t < NUM_TYPES; t++)
        for (int c = 0; c < INITIAL_COUNT[t]; c++) a[n++] = t;
    word_stream ws;
    stream_init(&ws, seed, game_id, episode, player == 0 ? TAG_SETUP0 : TAG_SETUP1);
    for (int i = 39; i >= 1; i--) {
        int j = (int)bounded(stream_next(&ws), (uint32_t)(i + 1));
        int tmp = a[i];
        a[i] = a[j];
        a[j] = tmp;
    }
    memcpy(types_out, a, sizeof(a));
}

static void fresh_state(orc_state* st, uint64_t seed, uint32_t game_id, uint32_t episode) {
    uint32_t redraws = st->redraws;
    memset(st, 0, sizeof(*st));
    st->redraws = redraws;
    st->game_id = game_id;
    st->episode = episode;
    for (int s = 0; s < NSQ; s++) st->board[s] = is_lake(s) ? LAKE : EMPTY;
    for (int p = 0; p < 2; p++) {
        int types[40];
        shuffle_setup(seed, game_id, episode, p, types);
        for (int slot = 0; slot < 40; slot++) {
            int id = p * 40 + slot;
            int sq = p == 0 ? slot : 99 - slot;
            orc_piece* pc = &st->piece[id];
            memset(pc, 0, sizeof(*pc));
            pc->type = types[slot];
            pc->alive = 1;
            pc->death_square = -1;
            st->board[sq] = id;
        }
    }
}

/* Fresh game for (game_id, episode); with auto-reset a setup that is
 * already terminal is replaced by the next episode's setup. */
static void reset_game(orc_state* st, const orc_cfg* cfg, uint32_t game_id, uint32_t episode) {
    fresh_state(st, cfg->seed, game_id, episode);
    terminal_check(st, cfg, -1);
    while (st->done && cfg->auto_reset) {
        st->redraws++;
        fresh_state(st, cfg->seed, game_id, st->episode + 1);
        terminal_check(st, cfg, -1);
    }
}

/* ------------------------------------------------------------------ */
static unsigned hidden_or_type10(const orc_piece* p) {
    /* channel slot for threat/evade/adjacency targets: revealed Spy..Marshal -> type,
     * hidden -> 10 */
    return p->revealed ? (unsigned)p->type : 10u;
}

static unsigned hidden_or_type11(const orc_piece* p) {
    /* protection slots: revealed Spy..Marshal -> 0..9, revealed Bomb -> 10, hidden -> 12 */
    if (!p->revealed) return 12u;
    return p->type == BOMB ? 10u : (unsigned)p->type;
}

/* Move application with battle resolution and the history features of
 * App. C.1 (threats, evasions, active adjacency, deaths, protection).
 * Returns 1 if the action was applied, 0 if it was not legal. */
static int apply_action(orc_state* st, const orc_cfg* cfg, int action) {
    if (action < 0 || action >= 10000) return 0;
    int from = action / 100, to = action % 100;
    int p = st->ply & 1, q = 1 - p;
    unsigned char legal[10000];
    legal_actions(st, p, rules_of(cfg), legal);
    if (!legal[action]) return 0;

    int X = st->board[from];

    /* previous move, if any: its mover A and destination a */
    int A = -1, a = -1, prev_was_threat = 0;
    if (st->ring_count > 0) {
        int slot = (st->ply - 1) & (RING - 1);
        int pt = st->ring_to[slot];
        int id = st->board[pt];
        if (id >= 0 && owner_of(id) == q) {
            A = id;
            a = pt;
            int nb[4], nn = neighbours(a, nb);
            for (int i = 0; i < nn; i++) {
                int o = st->board[nb[i]];
                if (o >= 0 && owner_of(o) == p) prev_was_threat = 1;
            }
        }
    }

    /* 1. active adjacency, evaluated before the move: every movable piece of
     *    p adjacent to an enemy piece it could have attacked but did not */
    for (int x = 0; x < NSQ; x++) {
        int id = st->board[x];
        if (id < 0 || owner_of(id) != p) continue;
        if (!is_movable_type(st->piece[id].type)) continue;
        int nb[4], nn = neighbours(x, nb);
        for (int i = 0; i < nn; i++) {
            int y = nb[i];
            int e = st->board[y];
            if (e < 0 || owner_of(e) != q) continue;
            if (x == from && y == to) continue;
            const orc_piece* Y = &st->piece[e];
            if (Y->revealed && !is_movable_type(Y->type)) continue;
            st->piece[id].adj |= 1u << hidden_or_type10(Y);
        }
    }

    /* 2. evasion: the mover was threatened by A on the previous move and now
     *    moves to an empty square that is not adjacent to A */
    int target = st->board[to];
    if (A >= 0 && adjacent(from, a) && target == EMPTY && !adjacent(to, a) &&
        !(st->piece[A].revealed && !is_movable_type(st->piece[A].type)))
        st->piece[X].evade |= 1u << hidden_or_type10(&st->piece[A]);

    /* 3. resolve the move or battle */
    int battle = target >= 0;
    int flag_captured_by = -1;
    int attacker_alive = 1;
    if (!battle) {
        st->board[to] = X;
        st->board[from] = EMPTY;
    } else {
        int Y = target;
        orc_piece* px = &st->piece[X];
        orc_piece* py = &st->piece[Y];
        int rY = py->revealed;
        int res = orc_battle(px->type, py->type);
        px->revealed = 1;
        py->revealed = 1;
        if (py->type == FLAG) flag_captured_by = p;
        st->board[from] = EMPTY;
        if (res == BATTLE_ATTACKER) {
            st->board[to] = X;
            py->alive = 0;
            py->death_square = to;
            py->death_cause = !rY ? 6 : 4;
        } else if (res == BATTLE_DEFENDER) {
            attacker_alive = 0;
            px->alive = 0;
            px->death_square = to;
            px->death_cause = !rY ? 3 : 1;
        } else {
            attacker_alive = 0;
            st->board[to] = EMPTY;
            px->alive = 0;
            px->death_square = to;
            px->death_cause = !rY ? 3 : 2;
            py->alive = 0;
            py->death_square = to;
            py->death_cause = !rY ? 6 : 5;
        }
    }
    st->piece[X].moved = 1;
    /* a move of more than one square is public proof of a Scout (App. A) */
    if (!adjacent(from, to)) st->piece[X].long_move = 1;

    /* 5. threats made by the move: the mover, if it stands on `to`, against
     *    every adjacent enemy piece */
    if (attacker_alive) {
        int nb[4], nn = neighbours(to, nb);
        for (int i = 0; i < nn; i++) {
            int e = st->board[nb[i]];
            if (e < 0 || owner_of(e) != q) continue;
            const orc_piece* Y = &st->piece[e];
            if (Y->revealed && !is_movable_type(Y->type)) continue;
            st->piece[X].threat |= 1u << hidden_or_type10(Y);
        }
    }

    /* 6. protection: a non-battle reply to a threat by A, in which the mover
     *    becomes adjacent to a square next to A */
    if (!battle && A >= 0 && prev_was_threat) {
        int nb[4], nn = neighbours(a, nb);
        for (int i = 0; i < nn; i++) {
            int s = nb[i];
            if (is_lake(s)) continue;
            if (!adjacent(s, to)) continue;
            if (s == from || adjacent(s, from)) continue;
            int o = st->board[s];
            const orc_piece* pa = &st->piece[A];
            if (o >= 0 && owner_of(o) == p) {
                orc_piece* pc = &st->piece[X];
                orc_piece* pb = &st->piece[o];
                pc->prot |= 1u << hidden_or_type11(pb);
                pc->prot_against |= 1u << hidden_or_type11(pa);
                pb->been_by |= 1u << hidden_or_type11(pc);
                pb->been_against |= 1u << hidden_or_type11(pa);
            } else if (o == EMPTY) {
                st->piece[X].prot |= 1u << 11;
                st->piece[X].prot_against |= 1u << hidden_or_type11(pa);
            }
        }
    }

    /* the two-square record of the mover's side and the chase, tracked only
     * while their rules are on */
    if (cfg->two_square) two_square_update(st, p, X, from, to);
    if (cfg->chasing) chase_update(st, p, battle, from, to, A, a);

    /* 7-8. move history and counters */
    int slot = st->ply & (RING - 1);
    st->ring_from[slot] = from;
    st->ring_to[slot] = to;
    if (st->ring_count < RING) st->ring_count++;
    st->ply += 1;
    st->battleless = battle ? 0 : st->battleless + 1;

    terminal_check(st, cfg, flag_captured_by);
    return 1;
}

/* ------------------------------------------------------------------ */
/* Probability channels (App. C.1 channels 12-35): the chance that a hidden
 * piece of player w has type T when the hidden types are a uniformly random
 * assignment of w's remaining type multiset, constrained by every hard public
 * fact: a piece that has moved is neither Flag nor Bomb, and a piece seen
 * moving more than one square in one move is a Scout (App. A).  Such a piece
 * is a known Scout: it leaves the hidden set and the multiset.  Returned as
 * an exact rational for the pieces that stay unknown. */
typedef struct {
    int n[NUM_TYPES];   /* hidden multiset */
    int H, I, M, U;
} hidden_stats;

static void compute_hidden_stats(const orc_state* st, int w, hidden_stats* hs) {
    memset(hs, 0, sizeof(*hs));
    for (int t = 0; t < NUM_TYPES; t++) hs->n[t] = INITIAL_COUNT[t];
    for (int id = w * 40; id < w * 40 + 40; id++) {
        const orc_piece* p = &st->piece[id];
        if (!p->alive || p->revealed || p->long_move) {
            hs->n[p->type]--;           /* known type: revealed, dead, or a known Scout */
        } else {
            hs->H++;
            if (p->moved) hs->M++;
        }
    }
    hs->I = hs->n[FLAG] + hs->n[BOMB];
    hs->U = hs->H - hs->M;
}

static void hidden_prob(const hidden_stats* hs, int moved, int t, long* num, long* den) {
    int movable_slots = hs->H - hs->I;
    if (moved) {
        if (!is_movable_type(t)) { *num = 0; *den = 1; return; }
        *num = hs->n[t];
        *den = movable_slots;
        return;
    }
    if (!is_movable_type(t)) {
        *num = hs->n[t];
        *den = hs->U;
        return;
    }
    *num = (long)hs->n[t] * (hs->U - hs->I);
    *den = (long)hs->U * movable_slots;
}

/* round-half-up of 255*num/den, 0 when den == 0 */
static int quant255(long num, long den) {
    if (den == 0) return 0;
    return (int)((510 * num + den) / (2 * den));
}

/* exported for tests: exact probability numerator/denominator for a hidden
 * piece of player w with the given moved flag and candidate type */
void orc_hidden_prob(const orc_state* st, int w, int moved, int t, long* num, long* den) {
    hidden_stats hs;
    compute_hidden_stats(st, w, &hs);
    hidden_prob(&hs, moved, t, num, den);
}

/* ------------------------------------------------------------------ */
/* Information state of observer o (App. C): 456 board channels followed by
 * 32 recent-move channels, each a 10x10 plane in the observer's frame
 * (blue's view is the board rotated by 180 degrees).  uint8 values:
 * indicators are 1, probabilities and fractions are round(255*x), and move
 * planes hold +1 (0x01) at the destination and -1 (0xFF) at the source. */
static int frame(int o, int sq) { return o == 0 ? sq : 99 - sq; }

static void put(uint8_t* out, int ch, int sq_frame, uint8_t v) {
    out[ch * PLANE + sq_frame] = v;
}

static void encode(const orc_state* st, const orc_cfg* cfg, int o, uint8_t* out) {
    int z = 1 - o;
    memset(out, 0, NCHAN * PLANE);
    hidden_stats hs_own, hs_opp;
    compute_hidden_stats(st, o, &hs_own);
    compute_hidden_stats(st, z, &hs_opp);

    for (int s = 0; s < NSQ; s++) {
        int f = frame(o, s);
        int id = st->board[s];
        if (id == LAKE) continue;
        if (id == EMPTY) {
            put(out, 38, f, 1);                                     /* 38: empty */
            continue;
        }
        const orc_piece* P = &st->piece[id];
        int own = owner_of(id) == o;
        if (own) {
            put(out, P->type, f, 1);                                /* 0-11: own type */
            if (!P->revealed) put(out, 36, f, 1);                   /* 36: own hidden */
            if (P->moved) put(out, 39, f, 1);                       /* 39: own moved */
        } else {
            if (!P->revealed) put(out, 37, f, 1);                   /* 37: opponent hidden */
            if (P->moved) put(out, 40, f, 1);                       /* 40: opponent moved */
        }
        /* 12-23 (about the opponent's pieces) and 24-35 (about own pieces, from
         * the opponent's point of view) */
        int pbase = own ? 24 : 12;
        const hidden_stats* hs = own ? &hs_own : &hs_opp;
        if (P->revealed || P->long_move) {
            put(out, pbase + P->type, f, 255);                      /* known type */
        } else {
            for (int t = 0; t < NUM_TYPES; t++) {
                long num, den;
                hidden_prob(hs, P->moved, t, &num, &den);
                put(out, pbase + t, f, (uint8_t)quant255(num, den));
            }
        }
        /* 43-75 own / 76-108 opponent: threat, evasion, active adjacency */
        int hbase = own ? 43 : 76;
        for (int j = 0; j < 11; j++) {
            if (P->threat & (1u << j)) put(out, hbase + j, f, 1);
            if (P->evade & (1u << j)) put(out, hbase + 11 + j, f, 1);
            if (P->adj & (1u << j)) put(out, hbase + 22 + j, f, 1);
        }
        /* 251-302 own / 303-354 opponent: protection groups of 13 */
        int gbase = own ? 251 : 303;
        for (int j = 0; j < 13; j++) {
            if (P->prot & (1u << j)) put(out, gbase + j, f, 1);
            if (P->prot_against & (1u << j)) put(out, gbase + 13 + j, f, 1);
            if (P->been_by & (1u << j)) put(out, gbase + 26 + j, f, 1);
            if (P->been_against & (1u << j)) put(out, gbase + 39 + j, f, 1);
        }
        /* 355-454: start square of the piece on this square */
        put(out, 355 + frame(o, start_square(id)), f, 1);
    }

    /* 41-42: fraction of the move budget and of the k-move budget used */
    int v41 = quant255(st->ply, cfg->max_moves);
    int v42 = quant255(st->battleless, cfg->k_battleless);
    for (int f = 0; f < NSQ; f++) {
        put(out, 41, f, (uint8_t)v41);
        put(out, 42, f, (uint8_t)v42);
    }

    /* 109-250: captured pieces by start square and by death square x cause */
    for (int id = 0; id < NPIECES; id++) {
        const orc_piece* P = &st->piece[id];
        if (P->alive) continue;
        int own = owner_of(id) == o;
        int t = P->type;
        if (t == FLAG) continue;
        int slot11 = t == BOMB ? 10 : t;
        put(out, (own ? 109 : 120) + slot11, frame(o, start_square(id)), 1);
        if (t <= MARSHAL)
            put(out, (own ? 131 : 191) + 10 * (P->death_cause - 1) + t,
                frame(o, P->death_square), 1);
    }

    /* 456-487: the last 32 moves, most recent first (App. C.2) */
    for (int i = 0; i < st->ring_count && i < RING; i++) {
        int slot = (st->ply - 1 - i) & (RING - 1);
        put(out, 456 + i, frame(o, st->ring_to[slot]), 0x01);
        put(out, 456 + i, frame(o, st->ring_from[slot]), 0xFF);
    }
}

/* ------------------------------------------------------------------ */
/* Canonical state record: 1536 bytes, little-endian, the interchange format
 * of the public interface (header fields at 0-23, per-player two-square
 * state at 24 + 8p, chase length and chaser at 40-41, board at 64, move ring
 * at 164, four 32-bit words per piece id at 256 + 16 id), serialised here on
 * its own. */
#define REC_BYTES 1536

static void put_u32(uint8_t* b, int off, uint32_t v) {
    b[off] = (uint8_t)v;
    b[off + 1] = (uint8_t)(v >> 8);
    b[off + 2] = (uint8_t)(v >> 16);
    b[off + 3] = (uint8_t)(v >> 24);
}

static uint32_t get_u32(const uint8_t* b, int off) {
    return (uint32_t)b[off] | ((uint32_t)b[off + 1] << 8) | ((uint32_t)b[off + 2] << 16) |
           ((uint32_t)b[off + 3] << 24);
}

static void to_record(const orc_state* st, uint8_t* rec) {
    memset(rec, 0, REC_BYTES);
    put_u32(rec, 0, st->game_id);
    put_u32(rec, 4, st->episode);
    put_u32(rec, 8, (uint32_t)st->ply);
    put_u32(rec, 12, (uint32_t)st->battleless);
    rec[16] = (uint8_t)st->ring_count;
    rec[17] = (uint8_t)st->done;
    rec[18] = (uint8_t)(int8_t)st->outcome;
    rec[19] = (uint8_t)st->reason;
    put_u32(rec, 20, st->redraws);
    for (int p = 0; p < 2; p++) {
        uint8_t* t = rec + 24 + 8 * p;
        t[0] = (uint8_t)(st->ts_n[p] ? st->ts_piece[p] : 0);
        t[1] = (uint8_t)st->ts_n[p];
        for (int i = 0; i < st->ts_n[p]; i++) t[2 + i] = (uint8_t)st->ts_pos[p][i];
    }
    rec[40] = (uint8_t)st->chase_len;
    rec[41] = (uint8_t)st->chaser;
    for (int s = 0; s < NSQ; s++) rec[64 + s] = (uint8_t)(int8_t)st->board[s];
    for (int m = 0; m < RING; m++) {
        rec[164 + 2 * m] = (uint8_t)st->ring_from[m];
        rec[164 + 2 * m + 1] = (uint8_t)st->ring_to[m];
    }
    for (int id = 0; id < NPIECES; id++) {
        const orc_piece* p = &st->piece[id];
        uint32_t w0 = (uint32_t)p->type | ((uint32_t)p->alive << 4) |
                      ((uint32_t)p->revealed << 5) | ((uint32_t)p->moved << 6) |
                      ((uint32_t)p->death_cause << 7) |
                      ((uint32_t)(p->alive ? 127 : p->death_square) << 10) |
                      ((uint32_t)p->been_against << 17) | ((uint32_t)p->long_move << 30);
        uint32_t w1 = p->threat | (p->evade << 11);
        uint32_t w2 = p->adj | (p->prot << 11);
        uint32_t w3 = p->prot_against | (p->been_by << 13);
        int off = 256 + 16 * id;
        put_u32(rec, off, w0);
        put_u32(rec, off + 4, w1);
        put_u32(rec, off + 8, w2);
        put_u32(rec, off + 12, w3);
    }
}

static void from_record(orc_state* st, const uint8_t* rec) {
    memset(st, 0, sizeof(*st));
    st->game_id = get_u32(rec, 0);
    st->episode = get_u32(rec, 4);
    st->ply = (int)get_u32(rec, 8);
    st->battleless = (int)get_u32(rec, 12);
    st->ring_count = rec[16];
    st->done = rec[17];
    st->outcome = (int8_t)rec[18];
    st->reason = rec[19];
    st->redraws = get_u32(rec, 20);
    for (int p = 0; p < 2; p++) {
        const uint8_t* t = rec + 24 + 8 * p;
        st->ts_piece[p] = t[0];
        st->ts_n[p] = t[1];
        for (int i = 0; i < 4; i++) st->ts_pos[p][i] = i < t[1] ? t[2 + i] : 0;
    }
    st->chase_len = rec[40];
    st->chaser = rec[41];
    for (int s = 0; s < NSQ; s++) st->board[s] = (int8_t)rec[64 + s];
    for (int m = 0; m < RING; m++) {
        st->ring_from[m] = rec[164 + 2 * m];
        st->ring_to[m] = rec[164 + 2 * m + 1];
    }
    for (int id = 0; id < NPIECES; id++) {
        int off = 256 + 16 * id;
        uint32_t w0 = get_u32(rec, off), w1 = get_u32(rec, off + 4);
        uint32_t w2 = get_u32(rec, off + 8), w3 = get_u32(rec, off + 12);
        orc_piece* p = &st->piece[id];
        p->type = (int)(w0 & 15);
        p->alive = (int)((w0 >> 4) & 1);
        p->revealed = (int)((w0 >> 5) & 1);
        p->moved = (int)((w0 >> 6) & 1);
        p->death_cause = (int)((w0 >> 7) & 7);
        int dsq = (int)((w0 >> 10) & 127);
        p->death_square = p->alive ? -1 : dsq;
        p->been_against = (w0 >> 17) & 0x1FFF;
        p->long_move = (int)((w0 >> 30) & 1);
        p->threat = w1 & 0x7FF;
        p->evade = (w1 >> 11) & 0x7FF;
        p->adj = w2 & 0x7FF;
        p->prot = (w2 >> 11) & 0x1FFF;
        p->prot_against = w3 & 0x1FFF;
        p->been_by = (w3 >> 13) & 0x1FFF;
    }
}

/* ------------------------------------------------------------------ */
/* Search-shaped resampling: draw the hidden types of player z uniformly
 * among assignments consistent with public information (revealed and dead
 * pieces known; a piece seen moving more than one square is a Scout; a piece
 * that moved is neither Flag nor Bomb).  Stands in
 * for the belief-model samples that search materialises on device (paper
 * section 2.5 and App. B reset behaviour). */
static void resample(const orc_state* src, orc_state* dst, uint64_t seed, uint32_t new_game_id) {
    *dst = *src;
    dst->game_id = new_game_id;
    int z = 1 - (src->ply & 1);
    hidden_stats hs;
    compute_hidden_stats(src, z, &hs);
    int unmoved[40], nu = 0;
    int assigned[NPIECES];
    for (int i = 0; i < NPIECES; i++) assigned[i] = -1;
    for (int id = z * 40; id < z * 40 + 40; id++) {
        const orc_piece* p = &src->piece[id];
        if (p->alive && !p->revealed && !p->moved) unmoved[nu++] = id;
    }
    word_stream ws;
    stream_init(&ws, seed, new_game_id, src->episode, TAG_RESAMPLE);
    /* step 1: positions of the hidden Flag and Bombs among unmoved pieces */
    int I = hs.I;
    for (int i = 0; i < I; i++) {
        int j = i + (int)bounded(stream_next(&ws), (uint32_t)(nu - i));
        int tmp = unmoved[i];
        unmoved[i] = unmoved[j];
        unmoved[j] = tmp;
    }
    for (int i = 0; i < I; i++) assigned[unmoved[i]] = (i < hs.n[FLAG]) ? FLAG : BOMB;
    /* step 2: the movable multiset shuffled over the remaining hidden pieces
     * in ascending id order */
    int list[40], L = 0;
    for (int t = 0; t <= MARSHAL; t++)
        for (int c = 0; c < hs.n[t]; c++) list[L++] = t;
    for (int i = L - 1; i >= 1; i--) {
        int j = (int)bounded(stream_next(&ws), (uint32_t)(i + 1));
        int tmp = list[i];
        list[i] = list[j];
        list[j] = tmp;
    }
    int k = 0;
    for (int id = z * 40; id < z * 40 + 40; id++) {
        const orc_piece* p = &src->piece[id];
        if (!p->alive || p->revealed || p->long_move) continue;
        if (assigned[id] >= 0) continue;
        assigned[id] = list[k++];
    }
    for (int id = z * 40; id < z * 40 + 40; id++)
        if (assigned[id] >= 0) dst->piece[id].type = assigned[id];
}

/* ------------------------------------------------------------------ */
/* Batch entry points (games are independent; OpenMP over games). */
size_t orc_state_bytes(void) { return sizeof(orc_state); }
int orc_record_bytes(void) { return REC_BYTES; }

void orc_batch_reset(orc_state* s, int n, const orc_cfg* cfg, const uint32_t* game_ids) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; i++) {
        s[i].redraws = 0;
        reset_game(&s[i], cfg, game_ids[i], 0);
    }
}

static int mask_one(const orc_state* st, const orc_cfg* cfg, uint64_t* mask) {
    unsigned char legal[10000];
    memset(mask, 0, MASK_WORDS * sizeof(uint64_t));
    if (st->done) return 0;
    int n = legal_actions(st, st->ply & 1, rules_of(cfg), legal);
    for (int a = 0; a < 10000; a++)
        if (legal[a]) mask[a >> 6] |= (uint64_t)1 << (a & 63);
    return n;
}

void orc_batch_mask(const orc_state* s, int n, const orc_cfg* cfg, uint64_t* mask, int16_t* num_legal) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; i++) {
        int c = mask_one(&s[i], cfg, mask + (size_t)i * MASK_WORDS);
        if (num_legal) num_legal[i] = (int16_t)c;
    }
}

/* Uniform legal action (App. B "SampleRandomLegalAction"): the r-th legal
 * action in ascending id order, r = bounded(Philox(seed; game, ply,
 * episode, MOVE).x, n). */
static int mask_bit(const uint64_t* mask, int a) { return (int)((mask[a >> 6] >> (a & 63)) & 1); }

/* Legal moves of the piece on square x in a mask (its actions 100x..100x+99). */
static int moves_from(const uint64_t* mask, int x) {
    int m = 0;
    for (int y = 0; y < NSQ; y++) m += mask_bit(mask, 100 * x + y);
    return m;
}

static int sample_one(const orc_state* st, const orc_cfg* cfg, const uint64_t* mask, int n) {
    if (n <= 0 || st->done) return -1;
    uint32_t w[4];
    philox_block(cfg->seed, st->game_id, (uint32_t)st->ply, st->episode, TAG_MOVE, w);
    if (cfg->sampler == SAMPLER_MAGNET) {
        /* the magnet policy (section 2.4, App. D.4: a movable piece uniformly at
         * random, then one of its legal moves uniformly at random): the
         * r1-th piece with a legal move in ascending square order, r1 =
         * bounded(y, P), then its r2-th move in ascending destination order,
         * r2 = bounded(z, m) */
        int P = 0;
        for (int x = 0; x < NSQ; x++) P += moves_from(mask, x) > 0;
        int r1 = (int)bounded(w[1], (uint32_t)P);
        for (int x = 0; x < NSQ; x++) {
            int m = moves_from(mask, x);
            if (m == 0) continue;
            if (r1-- > 0) continue;
            int r2 = (int)bounded(w[2], (uint32_t)m);
            for (int y = 0; y < NSQ; y++)
                if (mask_bit(mask, 100 * x + y) && r2-- == 0) return 100 * x + y;
        }
        return -1;
    }
    int r = (int)bounded(w[0], (uint32_t)n);
    for (int a = 0; a < 10000; a++) {
        if (mask_bit(mask, a)) {
            if (r == 0) return a;
            r--;
        }
    }
    return -1;
}

void orc_batch_sample(const orc_state* s, int n, const orc_cfg* cfg, const uint64_t* mask,
                      const int16_t* num_legal, int16_t* actions) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; i++)
        actions[i] = (int16_t)sample_one(&s[i], cfg, mask + (size_t)i * MASK_WORDS, num_legal[i]);
}

/* Step one game.  Output convention: done=1 with the finished episode's
 * outcome, reason and length when the game is (or becomes) terminal;
 * zeros otherwise.  Returns 0 on success, -1 for an illegal action. */
static int step_one(orc_state* st, const orc_cfg* cfg, int action, int8_t* done,
                    int8_t* outcome, uint8_t* reason, int16_t* ep_len) {
    if (st->done) {
        /* already terminal before this call: report it; with auto-reset the
         * game restarts with the next episode */
        *done = 1;
        *outcome = (int8_t)st->outcome;
        *reason = (uint8_t)st->reason;
        *ep_len = (int16_t)st->ply;
        if (cfg->auto_reset) reset_game(st, cfg, st->game_id, st->episode + 1);
        return 0;
    }
    if (action == -1) {
        *done = 0;
        *outcome = 0;
        *reason = 0;
        *ep_len = 0;
        return 0;
    }
    if (!apply_action(st, cfg, action)) {
        *done = 0;
        *outcome = 0;
        *reason = 0;
        *ep_len = 0;
        return -1;
    }
    if (st->done) {
        *done = 1;
        *outcome = (int8_t)st->outcome;
        *reason = (uint8_t)st->reason;
        *ep_len = (int16_t)st->ply;
        if (cfg->auto_reset) reset_game(st, cfg, st->game_id, st->episode + 1);
    } else {
        *done = 0;
        *outcome = 0;
        *reason = 0;
        *ep_len = 0;
    }
    return 0;
}

int orc_batch_step(orc_state* s, int n, const orc_cfg* cfg, const int16_t* actions,
                   int8_t* done, int8_t* outcome, uint8_t* reason, int16_t* ep_len) {
    int first_bad = -1;
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; i++) {
        if (step_one(&s[i], cfg, actions[i], &done[i], &outcome[i], &reason[i], &ep_len[i]) != 0) {
#pragma omp critical
            {
                if (first_bad < 0 || i < first_bad) first_bad = i;
            }
        }
    }
    return first_bad;
}

/* Both observers, or only the acting player (cfg->acting_obs: the
 * ComputeInfostateTensor of App. B.1 is the acting player's). */
static void encode_game(const orc_state* st, const orc_cfg* cfg, uint8_t* out) {
    if (cfg->acting_obs) {
        encode(st, cfg, st->ply & 1, out);
        return;
    }
    for (int o = 0; o < 2; o++) encode(st, cfg, o, out + (size_t)o * NCHAN * PLANE);
}

static size_t obs_per_game(const orc_cfg* cfg) { return (size_t)(cfg->acting_obs ? 1 : 2) * NCHAN * PLANE; }

void orc_batch_encode(const orc_state* s, int n, const orc_cfg* cfg, uint8_t* obs) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n; i++) encode_game(&s[i], cfg, obs + (size_t)i * obs_per_game(cfg));
}

/* Encode only selected games (index list) into a compact output. */
void orc_batch_encode_subset(const orc_state* s, const int32_t* idx, int m, const orc_cfg* cfg,
                             uint8_t* obs) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < m; i++) encode_game(&s[idx[i]], cfg, obs + (size_t)i * obs_per_game(cfg));
}

void orc_batch_export(const orc_state* s, int n, uint8_t* rec) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) to_record(&s[i], rec + (size_t)i * REC_BYTES);
}

void orc_batch_import(orc_state* s, int n, const uint8_t* rec) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) from_record(&s[i], rec + (size_t)i * REC_BYTES);
}

/* dst[i*per + j] = resample of src[i] with game id base + i*per + j */
void orc_batch_resample(const orc_state* src, int nsrc, int per, uint64_t seed,
                        uint32_t game_id_base, orc_state* dst) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int k = 0; k < nsrc * per; k++) {
        int i = k / per;
        resample(&src[i], &dst[k], seed, game_id_base + (uint32_t)k);
    }
}

/* One whole ply of the fused engine for every game: mask, sample, encode
 * both observers (of the pre-move state), then step with the configured
 * auto-reset.  Any output pointer may be NULL. */
void orc_batch_ply(orc_state* s, int n, const orc_cfg* cfg, uint64_t* mask, int16_t* num_legal,
                   int16_t* actions, uint8_t* obs, int8_t* done, int8_t* outcome,
                   uint8_t* reason, int16_t* ep_len) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n; i++) {
        uint64_t m[MASK_WORDS];
        int c = mask_one(&s[i], cfg, m);
        int a = sample_one(&s[i], cfg, m, c);
        if (mask) memcpy(mask + (size_t)i * MASK_WORDS, m, sizeof(m));
        if (num_legal) num_legal[i] = (int16_t)c;
        if (actions) actions[i] = (int16_t)a;
        if (obs) encode_game(&s[i], cfg, obs + (size_t)i * obs_per_game(cfg));
        int8_t d, oc;
        uint8_t r;
        int16_t el;
        step_one(&s[i], cfg, a, &d, &oc, &r, &el);
        if (done) done[i] = d;
        if (outcome) outcome[i] = oc;
        if (reason) reason[i] = r;
        if (ep_len) ep_len[i] = el;
    }
}

/* ------------------------------------------------------------------ */
/* Policies over the legal list (sections 2.4-2.5, App. D.7).  A game's legal list
 * is its legal actions in ascending order, padded to MAX_LEGAL with -1.    */
#define MAX_LEGAL 256

void orc_batch_legal_list(const orc_state* s, int n, const orc_cfg* cfg, int16_t* actions,
                          int16_t* num_legal) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; i++) {
        uint64_t m[MASK_WORDS];
        int c = mask_one(&s[i], cfg, m), k = 0;
        int16_t* out = actions + (size_t)i * MAX_LEGAL;
        for (int a = 0; a < 10000; a++)
            if (mask_bit(m, a)) out[k++] = (int16_t)a;
        for (; k < MAX_LEGAL; k++) out[k] = -1;
        num_legal[i] = (int16_t)c;
    }
}

/* The magnet policy rho over the legal list: 1 / (P * m), P pieces with a
 * legal move, m the moves of the listed action's piece (one IEEE single
 * division); 0 on padding. */
void orc_batch_magnet(const orc_state* s, int n, const orc_cfg* cfg, float* probs) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; i++) {
        uint64_t m[MASK_WORDS];
        mask_one(&s[i], cfg, m);
        int P = 0, k = 0;
        for (int x = 0; x < NSQ; x++) P += moves_from(m, x) > 0;
        float* out = probs + (size_t)i * MAX_LEGAL;
        for (int a = 0; a < 10000; a++)
            if (mask_bit(m, a)) out[k++] = 1.0f / (float)(P * moves_from(m, a / 100));
        for (; k < MAX_LEGAL; k++) out[k] = 0.0f;
    }
}

/* The search policy of App. D.7: the maximiser of <q, pi> - alpha KL(pi, rho)
 * - beta KL(pi, pi_theta), i.e. pi proportional to
 * [exp(q) rho^alpha pi_theta^beta]^(1/(alpha+beta)), over the legal list, in
 * double precision.  q and logpi (log pi_theta) are given per listed action. */
void orc_batch_mmd(const orc_state* s, int n, const orc_cfg* cfg, const float* q, const float* logpi,
                   double alpha, double beta, double* out) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; i++) {
        uint64_t m[MASK_WORDS];
        int c = mask_one(&s[i], cfg, m);
        int P = 0;
        for (int x = 0; x < NSQ; x++) P += moves_from(m, x) > 0;
        double e[MAX_LEGAL];
        double top = -1e300, sum = 0.0;
        int k = 0;
        for (int a = 0; a < 10000; a++) {
            if (!mask_bit(m, a)) continue;
            double rho = 1.0 / ((double)P * (double)moves_from(m, a / 100));
            size_t j = (size_t)i * MAX_LEGAL + k;
            e[k] = ((double)q[j] + alpha * log(rho) + beta * (double)logpi[j]) / (alpha + beta);
            if (e[k] > top) top = e[k];
            k++;
        }
        for (k = 0; k < c; k++) { e[k] = exp(e[k] - top); sum += e[k]; }
        double* o = out + (size_t)i * MAX_LEGAL;
        for (k = 0; k < MAX_LEGAL; k++) o[k] = k < c ? e[k] / sum : 0.0;
    }
}

/* Sample from a caller distribution over the legal list: u = the top 24
 * bits of word x of Philox(seed; game, ply, episode, POLICY) as a fraction;
 * the first listed action whose single-precision running sum (in list
 * order) exceeds u times the single-precision total; the last action with a
 * positive weight if rounding leaves none. */
void orc_batch_sample_policy(const orc_state* s, int n, const orc_cfg* cfg, const float* probs,
                             int16_t* actions) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; i++) {
        uint64_t m[MASK_WORDS];
        int c = mask_one(&s[i], cfg, m);
        int list[MAX_LEGAL], k = 0;
        for (int a = 0; a < 10000; a++)
            if (mask_bit(m, a)) list[k++] = a;
        const float* p = probs + (size_t)i * MAX_LEGAL;
        int pick = -1;
        if (c > 0 && !s[i].done) {
            uint32_t w[4];
            philox_block(cfg->seed, s[i].game_id, (uint32_t)s[i].ply, s[i].episode, TAG_POLICY, w);
            float total = 0.0f;
            for (k = 0; k < c; k++) total += p[k];
            float t = (float)(w[0] >> 8) * (1.0f / 16777216.0f) * total;
            float run = 0.0f;
            for (k = 0; k < c; k++) {
                run += p[k];
                if (p[k] > 0.0f) pick = list[k];
                if (run > t && p[k] > 0.0f) break;
            }
        }
        actions[i] = (int16_t)pick;
    }
}

/* Threads the batch entry points use (OpenMP), for reporting. */
#ifdef _OPENMP
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
#else
int orc_num_threads(void) { return 1; }
#endif

/* Single-game helpers for tests. */
int orc_legal_list(const orc_state* st, int player, int rules, unsigned char* legal10000) {
    return legal_actions(st, player, rules, legal10000);
}

int orc_has_legal_move(const orc_state* st, int player, int rules) {
    return has_legal_move(st, player, rules);
}

/* App. B.1 ComputeTwoSquareRuleApplies: the rule is on and removes at least
 * one move the acting player could otherwise make. */
int orc_two_square_applies(const orc_state* st, const orc_cfg* cfg) {
    if (!cfg->two_square || st->done) return 0;
    int p = st->ply & 1, r = rules_of(cfg);
    return legal_actions(st, p, r & ~RULE_TWO_SQUARE, NULL) != legal_actions(st, p, r, NULL);
}

/* The continuous-chasing rule is on and removes at least one move the acting
 * player could otherwise make. */
int orc_chase_applies(const orc_state* st, const orc_cfg* cfg) {
    if (!cfg->chasing || st->done) return 0;
    int p = st->ply & 1, r = rules_of(cfg);
    return legal_actions(st, p, r & ~RULE_CHASING, NULL) != legal_actions(st, p, r, NULL);
}

void orc_terminal_check(orc_state* st, const orc_cfg* cfg) { terminal_check(st, cfg, -1); }

void orc_setup_types(uint64_t seed, uint32_t game_id, uint32_t episode, int player,
                     int32_t* types40) {
    int t[40];
    shuffle_setup(seed, game_id, episode, player, t);
    for (int i = 0; i < 40; i++) types40[i] = t[i];
}

/* 64-bit FNV-1a over a byte buffer (used to compare large outputs). */
uint64_t orc_fnv1a64(const uint8_t* buf, size_t len) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < len; i++) {
        h ^= buf[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

/* Test support, not part of the method: a 64-bit digest of each of `count`
 * consecutive blocks of `block` bytes, the sum over the block of byte i times
 * w(i) modulo 2^64, where w(i) is the SplitMix64 output for the counter value
 * i + 1 (Steele, Lea and Flood, OOPSLA 2014).  Pseudo-random weights make
 * distinct blocks collide only by chance.  The tests form the same sum on the
 * device, so that observations can be compared without copying them out. */
static uint64_t digest_weight(uint64_t i) {
    uint64_t z = (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void orc_digest_blocks(const uint8_t* data, int64_t count, int64_t block, uint64_t* out) {
    uint64_t* w = (uint64_t*)malloc((size_t)block * sizeof(uint64_t));
    if (!w) return;
    for (int64_t i = 0; i < block; i++) w[i] = digest_weight((uint64_t)i);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < count; b++) {
        const uint8_t* p = data + b * block;
        uint64_t sum = 0;
        for (int64_t i = 0; i < block; i++) sum += (uint64_t)p[i] * w[i];
        out[b] = sum;
    }
    free(w);
}

/* Human-readable board (App. B "BoardStrs" debugging aid): rows 9..0 top to
 * bottom, three characters per square: owner ('r'/'b') and type symbol
 * (S 2-9 M F B), "~~" lake, ".." empty. */
void orc_board_string(const orc_state* st, char* out /* >= 311 bytes */) {
    static const char SYM[NUM_TYPES] = {'S', '2', '3', '4', '5', '6', '7', '8', '9', 'M', 'F', 'B'};
    int k = 0;
    for (int r = 9; r >= 0; r--) {
        for (int c = 0; c < 10; c++) {
            int id = st->board[r * 10 + c];
            if (id == LAKE) { out[k++] = '~'; out[k++] = '~'; }
            else if (id == EMPTY) { out[k++] = '.'; out[k++] = '.'; }
            else { out[k++] = owner_of(id) == 0 ? 'r' : 'b'; out[k++] = SYM[st->piece[id].type]; }
            out[k++] = c == 9 ? '\n' : ' ';
        }
    }
    out[k] = 0;
}
