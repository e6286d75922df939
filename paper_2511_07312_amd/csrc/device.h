// Device-side Stratego engine for gfx950: one wavefront (64 lanes) owns one
// game at a time.  The game's canonical record is staged in LDS; square-wise
// work maps lane l to squares l and l+64, piece-wise work to ids l and l+64,
// and scalar rule logic runs on lane 0 with wave-level fences in between.
//
// Paper: arXiv 2511.07312.  App. A (rules, Table "pieces"), App. B
// (simulator: ApplyActions, auto-reset, reset to non-initial states,
// SampleRandomLegalAction), App. C (information state), App. D.1 (k-move rule,
// maximum game length).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kSquares = 100;
constexpr int kPieces = 80;
constexpr int kChannels = 488;
constexpr int kObsPerObserver = kChannels * 100;  // 48800
constexpr int kObsPerGame = 2 * kObsPerObserver;  // 97600
constexpr int kMaskWords = 157;
constexpr int kRecordBytes = 1536;

// canonical record offsets
constexpr int kOffGameId = 0;
constexpr int kOffEpisode = 4;
constexpr int kOffPly = 8;
constexpr int kOffBattleless = 12;
constexpr int kOffRingCount = 16;
constexpr int kOffDone = 17;
constexpr int kOffOutcome = 18;
constexpr int kOffReason = 19;
constexpr int kOffRedraws = 20;
constexpr int kOffTwoSquare = 24;   // per player p at +8p: u8 piece, u8 n, u8 squares[4]
constexpr int kOffChaseLen = 40;    // u8 plies of the current chase (0 = none)
constexpr int kOffChaser = 41;      // u8 chasing player
constexpr int kOffBoard = 64;
constexpr int kOffRing = 164;
constexpr int kOffPieces = 256;

constexpr int kEmpty = -1;
constexpr int kLake = -2;

// piece types in the channel order of App. C.1 (channels 0-11)
constexpr int kSpy = 0, kScout = 1, kMiner = 2, kMarshal = 9, kFlag = 10, kBomb = 11;

// per-wave LDS slab
constexpr int kSlabProbQ = 1536;    // uint8 [owner][moved][type] quantised probabilities
constexpr int kSlabCounts = 1600;   // int32 [28]: known[2][12], hidden[2], moved_hidden[2]
constexpr int kSlabScratch = 1712;  // uint8 [80]: setup / resample work arrays
constexpr int kSlabImage = 1792;    // obs image segment (also holds the to-square sets)

// Observation staging layouts in LDS (the autotuner's "LDS layout" knob):
//   kLayoutBits (1): bit planes, one bit per output byte, both observers
//     staged at once (6.1 KB each) and expanded to bytes while streaming out;
//   2..6: byte images of both observers in 1, 2, 4, 8, 16 channel segments;
//   kLayoutBits1 (7): bit planes of one observer at a time (half the LDS of
//     layout 1, so twice the waves per CU, for a second pass over the pieces).
constexpr int kLayoutBits = 1;
constexpr int kLayoutBits1 = 7;
__host__ __device__ __forceinline__ constexpr bool valid_layout(int L) { return L >= 1 && L <= 7; }
__host__ __device__ __forceinline__ constexpr int segments_of(int L) { return L <= 1 ? 1 : 1 << (L - 2); }

// Channels per image segment (multiples of 4, so segments stay 16-byte aligned).
__host__ __device__ __forceinline__ constexpr int seg_channels_for(int segments) {
  return segments == 1 ? 488 : segments == 2 ? 244 : segments == 4 ? 124 : segments == 8 ? 64 : 32;
}
// Bytes of one observer's image segment; both observers' segments are staged.
__host__ __device__ __forceinline__ constexpr int seg_bytes_for(int segments) { return 100 * seg_channels_for(segments); }

// bit-plane layout: plane bit 100*c + f of observer o <=> byte (c, f) is 1 (or
// 255 / a table value in the special regions); move sources in a side plane
constexpr int kBitsPlane = 6112;                          // 48800 bits, padded
constexpr int kBitsMovePlane = 416;                       // 32 x 100 bits, padded
constexpr int kBitsPlane0 = kSlabImage;
constexpr int kBitsPlane1 = kBitsPlane0 + kBitsPlane;
constexpr int kBitsMove0 = kBitsPlane1 + kBitsPlane;
constexpr int kBitsMove1 = kBitsMove0 + kBitsMovePlane;
constexpr int kBitsCat0 = kBitsMove1 + kBitsMovePlane;    // uint8 [100] per observer
constexpr int kBitsCat1 = kBitsCat0 + 112;
constexpr int kBitsTab = kBitsCat1 + 112;                 // uint64 [2][24]
constexpr int kBitsSlabBytes = kBitsTab + 2 * 24 * 8;
// one-observer bit-plane layout
constexpr int kB1Plane = kSlabImage;
constexpr int kB1Move = kB1Plane + kBitsPlane;
constexpr int kB1Cat = kB1Move + kBitsMovePlane;          // uint8 [100]
constexpr int kB1Tab = kB1Cat + 112;                      // uint64 [24]
constexpr int kB1SlabBytes = kB1Tab + 24 * 8;

__host__ __device__ __forceinline__ constexpr int slab_bytes_for(int L) {
  return L == kLayoutBits ? kBitsSlabBytes : L == kLayoutBits1 ? kB1SlabBytes
                                           : kSlabImage + 2 * seg_bytes_for(segments_of(L));
}
// LDS bytes that must be zero when a game's encoding starts
__host__ __device__ __forceinline__ constexpr int image_bytes_for(int L) {
  return L == kLayoutBits ? kBitsCat0 - kSlabImage : L == kLayoutBits1 ? kB1Cat - kSlabImage
                                                   : 2 * seg_bytes_for(segments_of(L));
}

enum : int { kReasonNone = 0, kReasonFlag = 1, kReasonForcedWin = 2, kReasonForcedDraw = 3,
             kReasonKMove = 4, kReasonMaxMoves = 5 };

struct Rules {
  uint64_t seed;
  int32_t k_battleless;
  int32_t max_moves;
  int32_t auto_reset;
  int32_t two_square;   // enforce the two-square rule
  int32_t sampler;      // 0: uniform over legal actions; 1: magnet policy
  int32_t chasing;      // enforce the continuous-chasing rule
  int32_t acting_obs;   // encode only the acting player's information state
};

// Bytes of one game's observations: both observers, or the acting player's.
__host__ __device__ __forceinline__ int obs_bytes_per_game(const Rules& r) {
  return r.acting_obs ? kObsPerObserver : kObsPerGame;
}
enum : int { kSamplerUniform = 0, kSamplerMagnet = 1 };
constexpr int kMaxLegal = 256;   // legal-list capacity (at most 244 legal moves exist)

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// The lane id, made opaque where it is used: the empty asm statement hides the
// value from the optimiser, so that the many values derived from it (square
// numbers, neighbours, lane masks) are computed per game instead of being
// hoisted out of the per-game loop and kept live, and spilled, across it.
__device__ __forceinline__ int lane_here() {
  int l = lane_id();
  asm volatile("" : "+v"(l));
  return l;
}

// Order LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// A value every lane holds alike (read from LDS, say), moved to a scalar
// register so that the code using it runs on the scalar unit.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Inclusive prefix sum over the 64 lanes by DPP lane moves, which take no LDS
// round trip: Hillis-Steele steps of 1, 2, 4, 8 lanes inside each row of 16,
// then the totals of row 0 into row 1 and of row 2 into row 3 (lane 15 of a row
// to the next row), then lane 31's running total into rows 2 and 3.
__device__ __forceinline__ int dpp_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
  return v;
}

// ---------------------------------------------------------------- record access
__device__ __forceinline__ int board_at(const uint8_t* R, int s) { return (int8_t)R[kOffBoard + s]; }
__device__ __forceinline__ void set_board(uint8_t* R, int s, int v) { R[kOffBoard + s] = (uint8_t)(int8_t)v; }
__device__ __forceinline__ uint32_t* piece_words(uint8_t* R, int id) {
  return reinterpret_cast<uint32_t*>(R + kOffPieces + 16 * id);
}
__device__ __forceinline__ const uint32_t* piece_words(const uint8_t* R, int id) {
  return reinterpret_cast<const uint32_t*>(R + kOffPieces + 16 * id);
}
__device__ __forceinline__ uint32_t hdr_u32(const uint8_t* R, int off) {
  return *reinterpret_cast<const uint32_t*>(R + off);
}
__device__ __forceinline__ void set_hdr_u32(uint8_t* R, int off, uint32_t v) {
  *reinterpret_cast<uint32_t*>(R + off) = v;
}

// w0 fields: type 0-3, alive 4, revealed 5, moved 6, death cause 7-9,
// death square 10-16, been-protected-against 17-29, long move 30 (the piece
// once moved more than one square: App. A lets only a Scout do that, so its
// type is public although no battle revealed it)
__device__ __forceinline__ int p_type(uint32_t w0) { return w0 & 15; }
__device__ __forceinline__ bool p_alive(uint32_t w0) { return (w0 >> 4) & 1; }
__device__ __forceinline__ bool p_revealed(uint32_t w0) { return (w0 >> 5) & 1; }
__device__ __forceinline__ bool p_moved(uint32_t w0) { return (w0 >> 6) & 1; }
__device__ __forceinline__ bool p_long(uint32_t w0) { return (w0 >> 30) & 1; }
// the type is public: revealed in a battle, or a known Scout
__device__ __forceinline__ bool p_known(uint32_t w0) { return (w0 & ((1u << 5) | (1u << 30))) != 0; }
__device__ __forceinline__ int owner(int id) { return id >= 40 ? 1 : 0; }
__device__ __forceinline__ int start_sq(int id) { return id < 40 ? id : 139 - id; }
__device__ __forceinline__ bool movable_type(int t) { return t < kFlag; }

// threat / evasion / adjacency slot of a target piece: revealed Spy..Marshal
// -> its type, hidden -> 10; revealed Flag/Bomb -> -1 (no channel)
__device__ __forceinline__ int slot10(uint32_t w0) {
  if (!p_revealed(w0)) return 10;
  int t = p_type(w0);
  return t < kFlag ? t : -1;
}
// protection slot: revealed Spy..Marshal -> type, revealed Bomb -> 10, hidden -> 12
__device__ __forceinline__ int slot13(uint32_t w0) {
  if (!p_revealed(w0)) return 12;
  int t = p_type(w0);
  return t == kBomb ? 10 : t;
}

// x / 10 for 0 <= x < 1024 by a 24-bit multiply (full rate, where the
// compiler's division by a constant takes a quarter-rate 32-bit multiply)
__device__ __forceinline__ int div10(int x) { return (int)(__umul24((uint32_t)x, 205u) >> 11); }

__device__ __forceinline__ bool adjacent(int a, int b) {
  int ra = a / 10, ca = a - 10 * ra, rb = b / 10, cb = b - 10 * rb;
  int d = abs(ra - rb) + abs(ca - cb);
  return d == 1;
}

// orthogonal on-board neighbour k (0 up, 1 down, 2 left, 3 right) or -1
__device__ __forceinline__ int neighbour(int s, int k) {
  int r = div10(s), c = s - 10 * r;
  switch (k) {
    case 0: return r < 9 ? s + 10 : -1;
    case 1: return r > 0 ? s - 10 : -1;
    case 2: return c > 0 ? s - 1 : -1;
    default: return c < 9 ? s + 1 : -1;
  }
}

__device__ __forceinline__ bool is_lake_sq(int s) {
  int r = s / 10, c = s - 10 * r;
  return (r == 4 || r == 5) && (c == 2 || c == 3 || c == 6 || c == 7);
}

// ---------------------------------------------------------------- Philox4x32-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds of two 32x32
// multiplies with a Weyl key schedule.
__device__ __forceinline__ uint4 philox(uint4 c, uint64_t seed) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ uint32_t mulshift(uint32_t u, uint32_t n) {
  return (uint32_t)(((uint64_t)u * n) >> 32);
}

// sequential words x, y, z, w of blocks 0, 1, ... of one counter stream
struct WordStream {
  uint64_t seed;
  uint32_t id, episode, tag, block;
  uint4 buf;
  int used;
  __device__ void init(uint64_t s, uint32_t gid, uint32_t ep, uint32_t t) {
    seed = s; id = gid; episode = ep; tag = t; block = 0; used = 4;
  }
  __device__ uint32_t next() {
    if (used == 4) {
      buf = philox(make_uint4(id, block, episode, tag), seed);
      ++block;
      used = 0;
    }
    uint32_t v = used == 0 ? buf.x : used == 1 ? buf.y : used == 2 ? buf.z : buf.w;
    ++used;
    return v;
  }
};

// ---------------------------------------------------------------- global <-> LDS
__device__ __forceinline__ void load_record(uint8_t* R, const uint8_t* g) {
  const int lane = lane_id();
  const uint4* src = reinterpret_cast<const uint4*>(g);
  uint4* dst = reinterpret_cast<uint4*>(R);
  dst[lane] = src[lane];
  if (lane < 32) dst[64 + lane] = src[64 + lane];
  wave_sync();
}

__device__ __forceinline__ void store_record(uint8_t* g, const uint8_t* R) {
  const int lane = lane_id();
  const uint4* src = reinterpret_cast<const uint4*>(R);
  uint4* dst = reinterpret_cast<uint4*>(g);
  dst[lane] = src[lane];
  if (lane < 32) dst[64 + lane] = src[64 + lane];
}

// ---------------------------------------------------------------- legal moves
// Destinations of the piece on square x for player p as a 100-bit set (App. A:
// one orthogonal step to an empty or enemy square; Scouts any distance over
// empty squares, possibly ending on an enemy; no jumping over lakes or pieces;
// Flag and Bomb never move).
__device__ __forceinline__ void destinations(const uint8_t* R, int x, int p, uint64_t& lo,
                                             uint64_t& hi) {
  lo = 0;
  hi = 0;
  int id = board_at(R, x);
  if (id < 0 || owner(id) != p) return;
  int t = p_type(piece_words(R, id)[0]);
  if (!movable_type(t)) return;
  const int r = x / 10, c = x - 10 * r;
  const int reach = t == kScout ? 9 : 1;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int delta = d == 0 ? 10 : d == 1 ? -10 : d == 2 ? -1 : 1;
    const int room = d == 0 ? 9 - r : d == 1 ? r : d == 2 ? c : 9 - c;
    const int steps = room < reach ? room : reach;
    int y = x;
    for (int k = 0; k < steps; ++k) {
      y += delta;
      int o = board_at(R, y);
      if (o == kLake) break;
      bool enemy = o >= 0 && owner(o) != p;
      if (o == kEmpty || enemy) {
        if (y < 64) lo |= 1ull << y;
        else hi |= 1ull << (y - 64);
      }
      if (o != kEmpty) break;
    }
  }
}

// ---------------------------------------------------------------- two-square rule
// App. A (competitive play): a piece may not cross the same square boundary
// on more than three consecutive turns of its owner.  App. B.2: the record
// keeps, per player, the last-moved piece and up to four squares it occupied
// (oldest first, the last being its square).  A move along a row or column
// crosses the unit boundaries between consecutive squares of its segment.
struct Span { int axis, line, lo, hi; };   // boundaries lo..hi-1 of the line

__device__ __forceinline__ Span span_of(int u, int v) {
  const int ru = u / 10, cu = u - 10 * ru, rv = v / 10, cv = v - 10 * rv;
  Span sp;
  if (ru == rv) { sp.axis = 0; sp.line = ru; sp.lo = cu < cv ? cu : cv; sp.hi = cu < cv ? cv : cu; }
  else { sp.axis = 1; sp.line = cu; sp.lo = ru < rv ? ru : rv; sp.hi = ru < rv ? rv : ru; }
  return sp;
}

// The tracked piece of player p is restricted when it made the last three
// recorded moves of its side and they all crossed a common boundary: then
// returns true with its square x, the axis (0 row, 1 column) of their line,
// and the interval [L, H) of boundaries all three crossed.
__device__ __forceinline__ bool two_square_window(const uint8_t* R, int p, int& x, int& axis, int& L, int& H) {
  const uint8_t* t = R + kOffTwoSquare + 8 * p;
  x = t[5];
  if (t[1] != 4 || board_at(R, x) != (int)t[0]) return false;
  const Span a = span_of(t[2], t[3]), b = span_of(t[3], t[4]), c = span_of(t[4], t[5]);
  if (a.axis != b.axis || a.axis != c.axis || a.line != b.line || a.line != c.line) return false;
  axis = a.axis;
  L = max(a.lo, max(b.lo, c.lo));
  H = min(a.hi, min(b.hi, c.hi));
  return L < H;
}

// Does a move from x to y along the window's line cross a boundary in [L, H)?
__device__ __forceinline__ bool window_hit(int x, int y, int axis, int L, int H) {
  const int rx = x / 10, cx = x - 10 * rx, ry = y / 10, cy = y - 10 * ry;
  if (axis == 0 ? ry != rx : cy != cx) return false;
  const int u = axis == 0 ? cx : rx, v = axis == 0 ? cy : ry;
  return max(L, min(u, v)) < min(H, max(u, v));
}

// Does the rule forbid player p's move from -> to?
__device__ __forceinline__ bool two_square_forbids(const uint8_t* R, int p, int from, int to) {
  int x, axis, L, H;
  return two_square_window(R, p, x, axis, L, H) && x == from && window_hit(x, to, axis, L, H);
}

// Removes from the destination set (lo, hi) of the restricted piece's square
// the moves the rule forbids (only squares on the window's line can be hit).
__device__ __forceinline__ void two_square_clear(int x, int axis, int L, int H, uint64_t& lo, uint64_t& hi) {
  const int r = x / 10, c = x - 10 * r;
  for (int k = 0; k < 10; ++k) {
    const int y = axis == 0 ? 10 * r + k : 10 * k + c;
    if (y != x && window_hit(x, y, axis, L, H)) {
      if (y < 64) lo &= ~(1ull << y);
      else hi &= ~(1ull << (y - 64));
    }
  }
}

// After player p's piece X moved from -> to: extend its record when it is the
// same piece continuing from where it stopped, else start a new one; forget
// it when the piece did not end on `to`.  Single lane.
__device__ __forceinline__ void two_square_update(uint8_t* R, int p, int X, int from, int to) {
  uint8_t* t = R + kOffTwoSquare + 8 * p;
  const int n = t[1];
  if (board_at(R, to) != X) {
    for (int i = 0; i < 6; ++i) t[i] = 0;
  } else if (n > 0 && (int)t[0] == X && (int)t[1 + n] == from) {
    if (n == 4) { t[2] = t[3]; t[3] = t[4]; t[4] = t[5]; t[5] = (uint8_t)to; }
    else { t[2 + n] = (uint8_t)to; t[1] = (uint8_t)(n + 1); }
  } else {
    t[0] = (uint8_t)X; t[1] = 2; t[2] = (uint8_t)from; t[3] = (uint8_t)to; t[4] = 0; t[5] = 0;
  }
}

// ---------------------------------------------------------------- continuous-chasing rule
// App. A and Table "chase": a threat is a move after which the moved piece
// stands next to an enemy piece; an evasion moves a piece that the previous
// move threatened away from its threatener; a chase alternates threats by
// one player and evasions by the other.  The chasing player may not make a
// threat that recreates a position of the chase, unless the moved piece
// returns to the square it held before that player's previous turn.  The
// chase's positions (within the 32-ply move record; a position includes the
// side to move) are compared with the current one by their differences: undoing the chase's moves one by one,
// a position that differs from the current one in a single piece of the
// chaser, standing on square s, forbids that piece's move to s.
// Work area (per wave, 160 bytes of LDS): displaced pieces, their current
// squares, their squares in the rebuilt position, and the forbidden moves.
constexpr int kWorkPiece = 0, kWorkCur = 32, kWorkAt = 64, kWorkFrom = 96, kWorkTo = 128;

__device__ __forceinline__ bool chase_active(const uint8_t* R, int p) {
  const int L = R[kOffChaseLen];
  return L >= 2 && (L & 1) == 0 && R[kOffChaser] == p;
}

// Single lane: writes the forbidden (from, to) pairs to the work area and
// returns their number.
__device__ __forceinline__ int chase_forbidden_list(const uint8_t* R, int p, uint8_t* work) {
  if (!chase_active(R, p)) return 0;
  const int ply = (int)hdr_u32(R, kOffPly), rc = R[kOffRingCount], L = R[kOffChaseLen];
  const int K = L < rc ? L : rc;
  const int pslot = (ply - 2) & 31;
  const int prev_from = R[kOffRing + 2 * pslot], prev_to = R[kOffRing + 2 * pslot + 1];
  uint8_t* pc = work + kWorkPiece;
  uint8_t* cur = work + kWorkCur;
  uint8_t* at = work + kWorkAt;
  int ne = 0, ndiff = 0, nf = 0;
  for (int k = 1; k <= K; ++k) {
    const int slot = (ply - k) & 31;
    const int f = R[kOffRing + 2 * slot], g = R[kOffRing + 2 * slot + 1];
    int e = -1;
    for (int i = 0; i < ne; ++i)
      if (at[i] == g) { e = i; break; }
    if (e < 0) {   // the mover of that ply is still on g now
      const int id = board_at(R, g);
      if (id < 0) break;
      e = ne++;
      pc[e] = (uint8_t)id;
      cur[e] = (uint8_t)g;
      at[e] = (uint8_t)g;
    }
    ndiff -= at[e] != cur[e];
    at[e] = (uint8_t)f;
    ndiff += at[e] != cur[e];
    // a threat leaves the opponent to move: only positions an odd number of
    // plies back have the same side to move
    if (ndiff != 1 || (k & 1) == 0) continue;
    int x = -1, sq = -1, id = -1;
    for (int i = 0; i < ne; ++i)
      if (at[i] != cur[i]) { x = cur[i]; sq = at[i]; id = pc[i]; }
    if (owner(id) != p || (prev_to == x && prev_from == sq)) continue;
    bool threat = false;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int y = neighbour(sq, d);
      if (y < 0 || y == x) continue;
      const int o = board_at(R, y);
      if (o >= 0 && owner(o) != p) threat = true;
    }
    if (!threat) continue;
    work[kWorkFrom + nf] = (uint8_t)x;
    work[kWorkTo + nf] = (uint8_t)sq;
    ++nf;
  }
  return nf;
}

// Single lane, after player p's move from -> to (A: the previous move's
// mover still on its destination a, or -1): extend, restart or end the chase.
__device__ __forceinline__ void chase_update(uint8_t* R, int p, bool battle, int from, int to, int A, int a) {
  bool threat = false;
  if (!battle) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int y = neighbour(to, d);
      if (y < 0) continue;
      const int o = board_at(R, y);
      if (o >= 0 && owner(o) != p) threat = true;
    }
  }
  const bool evade = !battle && A >= 0 && adjacent(from, a) && !adjacent(to, a);
  int L = R[kOffChaseLen];
  const int C = R[kOffChaser];
  if (!battle && L > 0 && p == C && threat && (L & 1) == 0) ++L;
  else if (!battle && L > 0 && p != C && evade && (L & 1) == 1) ++L;
  else if (threat) { L = 1; R[kOffChaser] = (uint8_t)p; }
  else L = 0;
  R[kOffChaseLen] = (uint8_t)(L > 255 ? 255 : L);
  if (L == 0) R[kOffChaser] = 0;
}

// True when player p owns a movable piece with an adjacent empty or enemy
// square, i.e. p has at least one legal move (with the two-square rule, the
// tracked piece counts only through its allowed moves).
__device__ __forceinline__ bool has_move(const uint8_t* R, int p, Rules rules, uint8_t* work) {
  const int lane = lane_id();
  // the piece the two-square rule may restrict: it counts only through its
  // allowed moves (tested below); -1 when none
  const uint8_t* t = R + kOffTwoSquare + 8 * p;
  const int rx = __builtin_amdgcn_readfirstlane(rules.two_square && t[1] == 4 ? (int)t[5] : -1);
  if (rules.chasing && chase_active(R, p)) {
    // the chasing rule may forbid some threats: count the moves that remain
    int nf = 0;
    if (lane == 0) nf = chase_forbidden_list(R, p, work);
    nf = __shfl(nf, 0, 64);
    wave_sync();
    if (nf > 0) {
      int x2, axis, L, H;
      const bool window = rx >= 0 && two_square_window(R, p, x2, axis, L, H);
      bool any = false;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int x = lane + 64 * h;
        if (x >= kSquares) break;
        uint64_t lo, hi;
        destinations(R, x, p, lo, hi);
        if (window && x == rx) two_square_clear(x, axis, L, H, lo, hi);
        for (int i = 0; i < nf; ++i) {
          if (work[kWorkFrom + i] != x) continue;
          const int y = work[kWorkTo + i];
          if (y < 64) lo &= ~(1ull << y);
          else hi &= ~(1ull << (y - 64));
        }
        if (lo | hi) any = true;
      }
      return ballot(any) != 0;
    }
  }
  bool any = false;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int x = lane + 64 * h;
    if (x >= kSquares) break;
    if (x == rx) continue;
    int id = board_at(R, x);
    if (id < 0 || owner(id) != p || !movable_type(p_type(piece_words(R, id)[0]))) continue;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int y = neighbour(x, k);
      if (y < 0) continue;
      int o = board_at(R, y);
      if (o == kEmpty || (o >= 0 && owner(o) != p)) any = true;
    }
  }
  if (ballot(any) != 0) return true;
  if (rx < 0) return false;
  // a longer Scout move crosses the boundary next to rx that the one-square
  // move in its direction crosses, so the one-square moves decide
  int x, axis, L, H;
  const bool window = two_square_window(R, p, x, axis, L, H);
  bool some = false;
  if (lane < 4) {
    const int id = board_at(R, rx);
    const int y = neighbour(rx, lane);
    if (id >= 0 && owner(id) == p && movable_type(p_type(piece_words(R, id)[0])) && y >= 0) {
      const int o = board_at(R, y);
      some = (o == kEmpty || (o >= 0 && owner(o) != p)) && !(window && window_hit(rx, y, axis, L, H));
    }
  }
  return ballot(some) != 0;
}

// Direct test of one action against the movement rule (used to validate
// caller-supplied actions).
__device__ __forceinline__ bool action_is_legal(const uint8_t* R, int p, int action, bool two_square) {
  if (action < 0 || action >= 10000) return false;
  int from = action / 100, to = action - 100 * from;
  if (from == to) return false;
  int id = board_at(R, from);
  if (id < 0 || owner(id) != p) return false;
  int t = p_type(piece_words(R, id)[0]);
  if (!movable_type(t)) return false;
  int tgt = board_at(R, to);
  if (tgt == kLake || (tgt >= 0 && owner(tgt) == p)) return false;
  int rf = from / 10, cf = from - 10 * rf, rt = to / 10, ct = to - 10 * rt;
  if (rf != rt && cf != ct) return false;
  int dist = abs(rf - rt) + abs(cf - ct);
  if (t != kScout && dist != 1) return false;
  int stp = rf == rt ? (ct > cf ? 1 : -1) : (rt > rf ? 10 : -10);
  for (int y = from + stp; y != to; y += stp)
    if (board_at(R, y) != kEmpty) return false;
  return !(two_square && two_square_forbids(R, p, from, to));
}

// Mask words of the acting player: lane l returns words l, 64+l, 128+l (the
// last only for l < 29).  ts is the LDS array of 100 destination sets
// (2 x u64 each).  Returns the number of legal actions (wave-uniform).
__device__ __forceinline__ int legal_mask_words(const uint8_t* R, uint64_t* ts, uint64_t w[3], Rules rules,
                                                uint8_t* work) {
  const bool two_square = rules.two_square;
  const int lane = lane_id();
  const int p = hdr_u32(R, kOffPly) & 1;
  const bool done = R[kOffDone] != 0;
  int cnt = 0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int x = lane + 64 * h;
    if (x < kSquares) {
      uint64_t lo, hi;
      if (done) { lo = 0; hi = 0; }
      else destinations(R, x, p, lo, hi);
      ts[2 * x] = lo;
      ts[2 * x + 1] = hi;
      cnt += __popcll(lo) + __popcll(hi);
    }
  }
  if (lane == 0) { ts[200] = 0; ts[201] = 0; }   // sentinel set after square 99
  wave_sync();
  int rx, axis, L, H;
  if (two_square && !done && two_square_window(R, p, rx, axis, L, H)) {
    if (lane == 0) {
      uint64_t lo = ts[2 * rx], hi = ts[2 * rx + 1];
      const int before = __popcll(lo) + __popcll(hi);
      two_square_clear(rx, axis, L, H, lo, hi);
      ts[2 * rx] = lo;
      ts[2 * rx + 1] = hi;
      cnt -= before - (__popcll(lo) + __popcll(hi));
    }
    wave_sync();
  }
  if (rules.chasing && !done && chase_active(R, p)) {
    if (lane == 0) {
      const int nf = chase_forbidden_list(R, p, work);
      for (int i = 0; i < nf; ++i) {
        const int x = work[kWorkFrom + i], y = work[kWorkTo + i];
        uint64_t& set = ts[2 * x + (y >= 64)];
        const uint64_t bit = 1ull << (y & 63);
        if (set & bit) { set &= ~bit; --cnt; }
      }
    }
    wave_sync();
  }
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    int word = lane + 64 * g;
    uint64_t v = 0;
    if (word < kMaskWords) {
      int a0 = 64 * word;
      int f0 = a0 / 100;
      int off = a0 - 100 * f0;
      uint64_t lo = ts[2 * f0], hi = ts[2 * f0 + 1];
      v = off == 0 ? lo : off < 64 ? (lo >> off) | (hi << (64 - off)) : hi >> (off - 64);
      int rem = 100 - off;   // bits of set f0 that landed in this word
      if (rem < 64) v |= ts[2 * (f0 + 1)] << rem;
    }
    w[g] = v;
  }
  return wave_sum(cnt);
}

// k-th (0-based) set bit of a 64-bit word
__device__ __forceinline__ int select_bit(uint64_t w, int k) {
  int pos = 0;
  uint32_t v = (uint32_t)w;
  int c = __popc(v);
  if (k >= c) { k -= c; pos = 32; v = (uint32_t)(w >> 32); }
  c = __popc(v & 0xFFFFu);
  if (k >= c) { k -= c; pos += 16; v >>= 16; }
  c = __popc(v & 0xFFu);
  if (k >= c) { k -= c; pos += 8; v >>= 8; }
  c = __popc(v & 0xFu);
  if (k >= c) { k -= c; pos += 4; v >>= 4; }
  c = __popc(v & 0x3u);
  if (k >= c) { k -= c; pos += 2; v >>= 2; }
  c = v & 1u;
  if (k >= c) pos += 1;
  return pos;
}

// Uniform legal action from mask words held as in legal_mask_words.
__device__ __forceinline__ int sample_from_words(const uint64_t w[3], int n, uint64_t seed,
                                                 uint32_t game_id, uint32_t ply, uint32_t episode) {
  if (n <= 0) return -1;
  uint4 u = philox(make_uint4(game_id, ply, episode, 0u), seed);
  int r = (int)mulshift(u.x, (uint32_t)n);
  int base = 0;
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    int c = __popcll(w[g]);
    int incl = wave_incl_scan(c);
    int total = __shfl(incl, 63, 64);
    if (r < base + total) {
      uint64_t hit = ballot(base + incl > r);
      int L = __ffsll((unsigned long long)hit) - 1;
      int excl = __shfl(incl - c, L, 64);
      uint64_t word = __shfl(w[g], L, 64);
      int bit = select_bit(word, r - base - excl);
      return 64 * (64 * g + L) + bit;
    }
    base += total;
  }
  return -1;
}

// Magnet policy sample (section 2.4, App. D.4: a movable piece uniformly at
// random, then one of its legal moves uniformly at random).  (lo0, hi0) is
// the destination set of square lane, (lo1, hi1) that of square lane + 64
// (zero beyond 99).  Same Philox block as the uniform sampler: r1 =
// bounded(y, P) picks the r1-th square with a legal move in ascending
// order, r2 = bounded(z, m) its r2-th destination.  -1 without moves.
// draw() gives the block, and is called only when there is a legal move.
template <class Draw>
__device__ __forceinline__ int sample_magnet(uint64_t lo0, uint64_t hi0, uint64_t lo1, uint64_t hi1, Draw draw) {
  const int lane = lane_id();
  const uint64_t has0 = ballot((lo0 | hi0) != 0), has1 = ballot((lo1 | hi1) != 0);
  const int c0 = __popcll(has0), P = c0 + __popcll(has1);
  if (P == 0) return -1;
  const uint4 u = draw();
  const int r1 = (int)mulshift(u.y, (uint32_t)P);
  const int x = r1 < c0 ? select_bit(has0, r1) : 64 + select_bit(has1, r1 - c0);
  const int src = x & 63;
  const uint64_t lo = x < 64 ? __shfl(lo0, src, 64) : __shfl(lo1, src, 64);
  const uint64_t hi = x < 64 ? __shfl(hi0, src, 64) : __shfl(hi1, src, 64);
  const int nlo = __popcll(lo), m = nlo + __popcll(hi);
  const int r2 = (int)mulshift(u.z, (uint32_t)m);
  const int y = r2 < nlo ? select_bit(lo, r2) : 64 + select_bit(hi, r2 - nlo);
  (void)lane;
  return 100 * x + y;
}

__device__ __forceinline__ int sample_magnet(uint64_t lo0, uint64_t hi0, uint64_t lo1, uint64_t hi1,
                                             uint64_t seed, uint32_t game_id, uint32_t ply,
                                             uint32_t episode) {
  return sample_magnet(lo0, hi0, lo1, hi1, [&] { return philox(make_uint4(game_id, ply, episode, 0u), seed); });
}

// The 100-bit destination set of square x from packed mask words (global).
__device__ __forceinline__ void square_set_from_mask(const uint64_t* mask, int x, uint64_t& lo, uint64_t& hi) {
  lo = 0;
  hi = 0;
  if (x >= kSquares) return;
  const int a0 = 100 * x, w0 = a0 >> 6, off = a0 & 63;
  const uint64_t m0 = mask[w0], m1 = mask[w0 + 1], m2 = w0 + 2 < kMaskWords ? mask[w0 + 2] : 0ull;
  lo = off ? (m0 >> off) | (m1 << (64 - off)) : m0;
  hi = off ? (m1 >> off) | (m2 << (64 - off)) : m1;
  hi &= (1ull << 36) - 1;   // 100 - 64 bits
}

// ---------------------------------------------------------------- terminal check
// App. A: capture of the flag wins; a player to move without legal moves loses,
// a draw when neither side can move; App. D.1: k-move rule, maximum length.
// Priority: flag > no moves > k-move > max moves.  Writes done/outcome/reason.
__device__ __forceinline__ void terminal_check(uint8_t* R, Rules rules, int flag_winner, uint8_t* work) {
  const int ply = (int)hdr_u32(R, kOffPly);
  const int q = ply & 1;
  int done = 0, outcome = 0, reason = kReasonNone;
  if (flag_winner >= 0) {
    done = 1; outcome = flag_winner == 0 ? 1 : -1; reason = kReasonFlag;
  } else if (!has_move(R, q, rules, work)) {
    done = 1;
    if (!has_move(R, 1 - q, rules, work)) { outcome = 0; reason = kReasonForcedDraw; }
    else { outcome = (1 - q) == 0 ? 1 : -1; reason = kReasonForcedWin; }
  } else if ((int)hdr_u32(R, kOffBattleless) >= rules.k_battleless) {
    done = 1; reason = kReasonKMove;
  } else if (ply >= rules.max_moves) {
    done = 1; reason = kReasonMaxMoves;
  }
  if (lane_id() == 0) {
    R[kOffDone] = (uint8_t)done;
    R[kOffOutcome] = (uint8_t)(int8_t)outcome;
    R[kOffReason] = (uint8_t)reason;
  }
  wave_sync();
}

// ---------------------------------------------------------------- setup / reset
// type of the i-th element of the sorted initial multiset (Table "pieces":
// 1 Spy, 8 Scouts, 5 Miners, 4 Sergeants, 4 Lieutenants, 4 Captains, 3 Majors,
// 2 Colonels, 1 General, 1 Marshal, 1 Flag, 6 Bombs)
__device__ __forceinline__ int multiset_type(int i) {
  return i < 1 ? 0 : i < 9 ? 1 : i < 14 ? 2 : i < 18 ? 3 : i < 22 ? 4 : i < 26 ? 5
       : i < 29 ? 6 : i < 31 ? 7 : i < 32 ? 8 : i < 33 ? 9 : i < 34 ? 10 : 11;
}

__device__ __forceinline__ int initial_count(int t) {
  // 4 bits per type, Spy first: 1 8 5 4 4 4 3 2 1 1 1 6 (branch-free lookup)
  return (int)((0x611123444581ull >> (4 * t)) & 15u);
}

// Fresh uniformly random setup of both players for (game id, episode): a
// Durstenfeld shuffle of the multiset per player, red id i on square i, blue
// id 40+i on square 99-i.
__device__ __forceinline__ void fresh_setup(uint8_t* R, uint8_t* scratch, uint64_t seed, uint32_t game_id,
                            uint32_t episode, uint32_t redraws) {
  const int lane = lane_id();
  uint4* r4 = reinterpret_cast<uint4*>(R);
  r4[lane] = make_uint4(0, 0, 0, 0);
  if (lane < 32) r4[64 + lane] = make_uint4(0, 0, 0, 0);
  wave_sync();
  if (lane < 2) {
    uint8_t* a = scratch + 40 * lane;
    for (int i = 0; i < 40; ++i) a[i] = (uint8_t)multiset_type(i);
    WordStream ws;
    ws.init(seed, game_id, episode, 1u + (uint32_t)lane);
    for (int i = 39; i >= 1; --i) {
      int j = (int)mulshift(ws.next(), (uint32_t)(i + 1));
      uint8_t tmp = a[i];
      a[i] = a[j];
      a[j] = tmp;
    }
  }
  if (lane == 0) {
    set_hdr_u32(R, kOffGameId, game_id);
    set_hdr_u32(R, kOffEpisode, episode);
    set_hdr_u32(R, kOffRedraws, redraws);
  }
  wave_sync();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int s = lane + 64 * h;
    if (s < kSquares) {
      int v = kEmpty;
      if (is_lake_sq(s)) v = kLake;
      else if (s < 40) v = s;
      else if (s >= 60) v = 139 - s;
      set_board(R, s, v);
    }
    int id = lane + 64 * h;
    if (id < kPieces) {
      int t = scratch[id];   // id < 40: red slot id; id >= 40: blue slot id-40
      piece_words(R, id)[0] = (uint32_t)t | (1u << 4) | (127u << 10);
    }
  }
  wave_sync();
}

__device__ __forceinline__ void reset_game(uint8_t* R, uint8_t* scratch, uint8_t* work, Rules rules, uint32_t game_id,
                           uint32_t episode, uint32_t redraws) {
  // a fresh setup has no move history, so neither competitive rule can bite
  rules.two_square = 0;
  rules.chasing = 0;
  fresh_setup(R, scratch, rules.seed, game_id, episode, redraws);
  terminal_check(R, rules, -1, work);
  // A setup that is already terminal is replaced by the next episode's setup
  // (probability ~4e-6 per game); the bound only guards against a hang.
  int guard = 0;
  while (R[kOffDone] && rules.auto_reset && guard < 1000) {
    ++episode;
    ++redraws;
    ++guard;
    fresh_setup(R, scratch, rules.seed, game_id, episode, redraws);
    terminal_check(R, rules, -1, work);
  }
}

// ---------------------------------------------------------------- move application
// Applies a legal action of the player to move and updates the history
// features of App. C.1: active adjacency (attacks available but not taken,
// before the move), evasion (a piece threatened by the previous move steps
// to an empty square away from the threatener), battle resolution with
// reveal and death records, threats made by the mover, and protection (a
// non-battle reply to a threat in which the mover newly becomes adjacent to a
// square next to the threatener).  Then pushes the move into the ring,
// advances the counters and runs the terminal check.
__device__ __forceinline__ void apply_action(uint8_t* R, Rules rules, int action, uint8_t* work) {
  const int lane = lane_id();
  const int from = action / 100, to = action - 100 * (action / 100);
  const int ply = (int)hdr_u32(R, kOffPly);
  const int p = ply & 1, q = 1 - p;
  const int X = board_at(R, from);

  // previous move: its mover A (still standing on its destination a)
  int A = -1, a = -1;
  bool prev_threat = false;
  const int ring_count = R[kOffRingCount];
  if (ring_count > 0) {
    int slot = (ply - 1) & 31;
    int pt = R[kOffRing + 2 * slot + 1];
    int id = board_at(R, pt);
    if (id >= 0 && owner(id) == q) {
      A = id;
      a = pt;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        int y = neighbour(a, k);
        if (y < 0) continue;
        int o = board_at(R, y);
        if (o >= 0 && owner(o) == p) prev_threat = true;
      }
    }
  }

  // 1. active adjacency (pre-move), lane-parallel over squares
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int x = lane + 64 * h;
    if (x >= kSquares) break;
    int id = board_at(R, x);
    if (id < 0 || owner(id) != p) continue;
    if (!movable_type(p_type(piece_words(R, id)[0]))) continue;
    uint32_t bits = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int y = neighbour(x, k);
      if (y < 0) continue;
      int e = board_at(R, y);
      if (e < 0 || owner(e) != q) continue;
      if (x == from && y == to) continue;
      int sl = slot10(piece_words(R, e)[0]);
      if (sl >= 0) bits |= 1u << sl;
    }
    if (bits) piece_words(R, id)[2] |= bits;
  }
  wave_sync();

  int flag_winner = -1;
  if (lane == 0) {
    uint32_t* px = piece_words(R, X);
    const int tgt = board_at(R, to);
    // 2. evasion
    if (A >= 0 && adjacent(from, a) && tgt == kEmpty && !adjacent(to, a)) {
      const int sl = slot10(piece_words(R, A)[0]);
      if (sl >= 0) px[1] |= (1u << sl) << 11;
    }
    // 3-4. move or battle with death records
    const bool battle = tgt >= 0;
    bool attacker_alive = true;
    if (!battle) {
      set_board(R, to, X);
      set_board(R, from, kEmpty);
    } else {
      uint32_t* py = piece_words(R, tgt);
      const int ta = p_type(px[0]), td = p_type(py[0]);
      const bool rY = p_revealed(py[0]);
      int res;   // 0 attacker wins, 1 defender wins, 2 tie (Table "pieces")
      if (td == kFlag) res = 0;
      else if (td == kBomb) res = ta == kMiner ? 0 : 1;
      else if (ta == kSpy && td == kMarshal) res = 0;
      else res = ta > td ? 0 : ta < td ? 1 : 2;
      px[0] |= 1u << 5;
      py[0] |= 1u << 5;
      if (td == kFlag) flag_winner = p;
      set_board(R, from, kEmpty);
      const uint32_t clear = (1u << 4) | (7u << 7) | (127u << 10);
      if (res == 0) {
        set_board(R, to, X);
        py[0] = (py[0] & ~clear) | ((rY ? 4u : 6u) << 7) | ((uint32_t)to << 10);
      } else if (res == 1) {
        attacker_alive = false;
        px[0] = (px[0] & ~clear) | ((rY ? 1u : 3u) << 7) | ((uint32_t)to << 10);
      } else {
        attacker_alive = false;
        set_board(R, to, kEmpty);
        px[0] = (px[0] & ~clear) | ((rY ? 2u : 3u) << 7) | ((uint32_t)to << 10);
        py[0] = (py[0] & ~clear) | ((rY ? 5u : 6u) << 7) | ((uint32_t)to << 10);
      }
    }
    px[0] |= 1u << 6;   // moved
    if (!adjacent(from, to)) px[0] |= 1u << 30;   // a long move: a known Scout
    // 5. threats by the mover from its destination
    if (attacker_alive) {
      for (int k = 0; k < 4; ++k) {
        int y = neighbour(to, k);
        if (y < 0) continue;
        int e = board_at(R, y);
        if (e < 0 || owner(e) != q) continue;
        int sl = slot10(piece_words(R, e)[0]);
        if (sl >= 0) px[1] |= 1u << sl;
      }
    }
    // 6. protection
    if (!battle && A >= 0 && prev_threat) {
      const uint32_t wA = piece_words(R, A)[0];
      const uint32_t bitA = 1u << slot13(wA);
      for (int k = 0; k < 4; ++k) {
        int s = neighbour(a, k);
        if (s < 0 || is_lake_sq(s)) continue;
        if (!adjacent(s, to) || s == from || adjacent(s, from)) continue;
        int o = board_at(R, s);
        if (o >= 0 && owner(o) == p) {
          uint32_t* pb = piece_words(R, o);
          px[2] |= (1u << slot13(pb[0])) << 11;
          px[3] |= bitA;
          pb[3] |= (1u << slot13(px[0])) << 13;
          pb[0] |= bitA << 17;
        } else if (o == kEmpty) {
          px[2] |= (1u << 11) << 11;
          px[3] |= bitA;
        }
      }
    }
    // the two-square record of the mover's side and the chase (tracked only
    // while their rules are on)
    if (rules.two_square) two_square_update(R, p, X, from, to);
    if (rules.chasing) chase_update(R, p, battle, from, to, A, a);
    // 7-8. ring and counters
    const int slot = ply & 31;
    R[kOffRing + 2 * slot] = (uint8_t)from;
    R[kOffRing + 2 * slot + 1] = (uint8_t)to;
    if (ring_count < 32) R[kOffRingCount] = (uint8_t)(ring_count + 1);
    set_hdr_u32(R, kOffPly, (uint32_t)(ply + 1));
    set_hdr_u32(R, kOffBattleless, battle ? 0u : hdr_u32(R, kOffBattleless) + 1u);
  }
  flag_winner = __shfl(flag_winner, 0, 64);
  wave_sync();
  terminal_check(R, rules, flag_winner, work);
}

struct StepOut {
  int done, outcome, reason, ep_len;
  bool illegal;
};

// One ApplyActions step of one game (App. B).  Returns the per-game outputs.
// validate: check the action against the rules first (caller-supplied
// actions); actions drawn from the legal mask skip the check.
template <bool validate>
__device__ __forceinline__ StepOut step_game(uint8_t* R, uint8_t* scratch, uint8_t* work, Rules rules, int action) {
  StepOut o{0, 0, 0, 0, false};
  const bool was_done = R[kOffDone] != 0;
  if (!was_done) {
    if (action == -1) return o;
    if (validate) {
      const int p = hdr_u32(R, kOffPly) & 1;
      bool ok = action_is_legal(R, p, action, rules.two_square);
      if (ok && rules.chasing && chase_active(R, p)) {
        int nf = 0;
        if (lane_id() == 0) nf = chase_forbidden_list(R, p, work);
        nf = __shfl(nf, 0, 64);
        wave_sync();
        for (int i = 0; i < nf; ++i)
          if (work[kWorkFrom + i] == action / 100 && work[kWorkTo + i] == action % 100) ok = false;
      }
      if (!ok) {
        o.illegal = true;
        return o;
      }
    }
    apply_action(R, rules, action, work);
  }
  // a game that was over already, or ended now, reports its episode and,
  // with auto-reset, restarts with the next one
  if (R[kOffDone]) {
    o.done = 1;
    o.outcome = (int8_t)R[kOffOutcome];
    o.reason = R[kOffReason];
    o.ep_len = (int)hdr_u32(R, kOffPly);
    if (rules.auto_reset)
      reset_game(R, scratch, work, rules, hdr_u32(R, kOffGameId), hdr_u32(R, kOffEpisode) + 1,
                 hdr_u32(R, kOffRedraws));
  }
  return o;
}

// ---------------------------------------------------------------- register boards
// Fast path of the fused ply while neither competitive-play rule is on.  The
// game's squares sit in registers (lane l holds squares l and 64 + l: the
// piece id and that piece's word 0) and each player's pieces form wave-uniform
// 100-square sets built by ballots.  Legal destinations become bit tests on
// those sets, the no-move test of the terminal check set arithmetic, and a
// look-up at a square the whole wave agrees on a lane read (v_readlane)
// instead of a chain of dependent LDS loads.  The record in LDS stays the
// state and is written exactly as the general path writes it.
struct Set100 {
  uint64_t lo, hi;   // squares 0-63 in lo, squares 64-99 in bits 0-35 of hi
};
constexpr uint64_t kHi36 = (1ull << 36) - 1;

__host__ __device__ constexpr Set100 column_set(int c) {
  Set100 s{0, 0};
  for (int r = 0; r < 10; ++r) {
    const int x = 10 * r + c;
    if (x < 64) s.lo |= 1ull << x;
    else s.hi |= 1ull << (x - 64);
  }
  return s;
}
constexpr Set100 kCol0 = column_set(0), kCol9 = column_set(9);
constexpr Set100 kLakeSet = {(1ull << 42) | (1ull << 43) | (1ull << 46) | (1ull << 47) | (1ull << 52) |
                                 (1ull << 53) | (1ull << 56) | (1ull << 57),
                             0};
constexpr Set100 kAllSquares = {~0ull, kHi36};

__device__ __forceinline__ Set100 s_or(Set100 a, Set100 b) { return Set100{a.lo | b.lo, a.hi | b.hi}; }
__device__ __forceinline__ Set100 s_and(Set100 a, Set100 b) { return Set100{a.lo & b.lo, a.hi & b.hi}; }
__device__ __forceinline__ Set100 s_andnot(Set100 a, Set100 b) { return Set100{a.lo & ~b.lo, a.hi & ~b.hi}; }
__device__ __forceinline__ bool s_any(Set100 a) { return (a.lo | a.hi) != 0; }
__device__ __forceinline__ bool s_has(Set100 s, int y) {
  return ((y < 64 ? s.lo >> y : s.hi >> (y - 64)) & 1ull) != 0;
}
// each square y moved to y + 10, y - 10, y + 1 (same row) and y - 1 (same row)
__device__ __forceinline__ Set100 s_up(Set100 s) { return Set100{s.lo << 10, ((s.hi << 10) | (s.lo >> 54)) & kHi36}; }
__device__ __forceinline__ Set100 s_down(Set100 s) { return Set100{(s.lo >> 10) | (s.hi << 54), s.hi >> 10}; }
__device__ __forceinline__ Set100 s_right(Set100 s) {
  s = s_andnot(s, kCol9);
  return Set100{s.lo << 1, ((s.hi << 1) | (s.lo >> 63)) & kHi36};
}
__device__ __forceinline__ Set100 s_left(Set100 s) {
  s = s_andnot(s, kCol0);
  return Set100{(s.lo >> 1) | (s.hi << 63), s.hi >> 1};
}
// squares orthogonally next to a square of s
__device__ __forceinline__ Set100 s_nbrs(Set100 s) { return s_or(s_or(s_up(s), s_down(s)), s_or(s_left(s), s_right(s))); }

// The squares in registers: lane l holds squares l and 64 + l.
struct SquareRegs {
  int id[2];        // board entry of the square (kLake beyond square 99)
  uint32_t w0[2];   // word 0 of the piece there, 0 without one
  int tid[2];       // board entry of the square whose column-major index
                    // 10 * column + row is lane (resp. 64 + lane)
};

__device__ __forceinline__ Set100 ballot100(bool b0, bool b1) { return Set100{ballot(b0), ballot(b1) & kHi36}; }

__device__ __forceinline__ void load_regs(const uint8_t* R, SquareRegs& q) {
  const int lane = lane_here();
  q.id[0] = board_at(R, lane);
  q.id[1] = lane < kSquares - 64 ? board_at(R, 64 + lane) : kLake;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // column-major index t: column t / 10, row t % 10
    const int t = lane + 64 * h, tc = div10(t);
    q.tid[h] = t < kSquares ? board_at(R, 10 * (t - 10 * tc) + tc) : kLake;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) q.w0[h] = q.id[h] >= 0 ? piece_words(R, q.id[h])[0] : 0u;
}

// id names a piece of player p (ids 40p .. 40p + 39); false for -1 and -2
__device__ __forceinline__ bool owned_by(int id, int p) { return (unsigned)(id - 40 * p) < 40u; }

// Squares holding player p's pieces, and the empty squares.
__device__ __forceinline__ Set100 occupied(const SquareRegs& q, int p) {
  return ballot100(owned_by(q.id[0], p), owned_by(q.id[1], p));
}
__device__ __forceinline__ Set100 empty_set(const SquareRegs& q) {
  return ballot100(q.id[0] == kEmpty, q.id[1] == kEmpty);
}

// A register value at a square the whole wave agrees on.
__device__ __forceinline__ int reg_at(const int v[2], int y) {
  return __builtin_amdgcn_readlane(y < 64 ? v[0] : v[1], y & 63);
}
__device__ __forceinline__ uint32_t reg_at(const uint32_t v[2], int y) {
  return (uint32_t)__builtin_amdgcn_readlane((int)(y < 64 ? v[0] : v[1]), y & 63);
}

// 64 bits of a 100-square set starting at square s (0 <= s < 128; squares
// past 99 read as absent).
__device__ __forceinline__ uint64_t s_window(Set100 v, int s) {
  if (s >= 64) return v.hi >> (s - 64);
  return s == 0 ? v.lo : (v.lo >> s) | (v.hi << (64 - s));
}

// The 10 squares of a row (s = 10 * row) or, in a transposed set, of a column
// (s = 10 * column), as bits 0-9.
__device__ __forceinline__ uint32_t line10(Set100 v, int s) { return (uint32_t)s_window(v, s) & 1023u; }

// Moves of a Scout at position i of a 10-square line towards higher
// positions: the run of open squares after i, plus one if the square that
// ends it is a stop (an enemy) square; the line's end stops the run, since
// positions past 9 read as closed and as no stop.
__device__ __forceinline__ uint32_t line_up(uint32_t open, uint32_t stop, int i) {
  const int run = __builtin_ctz(~(open >> (i + 1)));
  return (uint32_t)run + ((stop >> (i + 1 + run)) & 1u);
}
// The same towards lower positions: bits i-1 .. 0 are moved to the top of the
// word, where the run is counted from bit 31 down.
__device__ __forceinline__ uint32_t line_down(uint32_t open, uint32_t stop, int i) {
  const uint32_t top = (open << 1) << (31 - i);   // bit i-1 to bit 31; nothing for i = 0
  const int run = __builtin_clz(~top);             // at most i: the low 32 - i bits of ~top are set
  const int below = i - 1 - run;                   // the square that ends the run
  return (uint32_t)run + (below >= 0 ? (stop >> (below & 31)) & 1u : 0u);
}

// Length of the run of squares of `open` going up from index i + 1 (at most
// room), and whether the square after it is in `stop` (a capture).
__device__ __forceinline__ int run_up(Set100 open, Set100 stop, int i, int room, int& cap) {
  int run = __builtin_ctzll(~s_window(open, i + 1));
  run = run < room ? run : room;
  cap = run < room && s_has(stop, i + 1 + run) ? 1 : 0;
  return run;
}
// The same going down from index i - 1 (room = squares below i in its line).
__device__ __forceinline__ int run_down(Set100 open, Set100 stop, int i, int room, int& cap) {
  if (room == 0) { cap = 0; return 0; }
  const uint64_t m = (1ull << room) - 1;
  const uint64_t gaps = ~s_window(open, i - room) & m;   // bit j: index i - room + j not open
  const int run = gaps == 0 ? room : room - 1 - (63 - __builtin_clzll(gaps));
  cap = run < room && s_has(stop, i - 1 - run) ? 1 : 0;
  return run;
}

// Destination sets of player p's pieces on the lane's two squares (App. A
// movement rules, as destinations()): d[0..1] for square lane, d[2..3] for
// square 64 + lane; all empty for a finished game.
__device__ __forceinline__ void fast_dests(const SquareRegs& q, int p, bool done, uint64_t d[4]) {
  const int lane = lane_here();
  const Set100 empty = empty_set(q);
  const Set100 target = s_or(empty, occupied(q, 1 - p));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int x = lane + 64 * h;
    uint64_t lo = 0, hi = 0;
    const int t = p_type(q.w0[h]);
    if (!done && owned_by(q.id[h], p) && movable_type(t)) {
      const int reach = t == kScout ? 9 : 1;
      const int r = x / 10, c = x - 10 * r;
#pragma unroll
      for (int dir = 0; dir < 4; ++dir) {
        const int delta = dir == 0 ? 10 : dir == 1 ? -10 : dir == 2 ? -1 : 1;
        const int room = dir == 0 ? 9 - r : dir == 1 ? r : dir == 2 ? c : 9 - c;
        const int steps = room < reach ? room : reach;
        int y = x;
        for (int k = 0; k < steps; ++k) {
          y += delta;
          if (!s_has(target, y)) break;
          if (y < 64) lo |= 1ull << y;
          else hi |= 1ull << (y - 64);
          if (!s_has(empty, y)) break;
        }
      }
    }
    d[2 * h] = lo;
    d[2 * h + 1] = hi;
  }
}

// Legal moves of player p's pieces on the lane's two squares as counts per
// direction, 4 bits each, in ascending order of destination: down (x - 10k,
// bits 0-3), left (x - k, 4-7), right (x + k, 8-11), up (x + 10k, 12-15); 0
// for other squares and in a finished game.  A piece other than a Scout
// steps to a neighbouring empty or enemy square (App. A): its four tests are
// bits of shifted copies of the target set.  A Scout runs over empty squares
// and may end on an enemy square: its run lengths come from bit scans of the
// empty squares, row-major along its row and column-major (the transposed
// sets) along its column.  Sampling needs only these counts, not the sets.
__device__ __forceinline__ int count_of(uint32_t pk) {
  return (int)((pk & 15u) + ((pk >> 4) & 15u) + ((pk >> 8) & 15u) + (pk >> 12));
}

__device__ __forceinline__ void dir_counts(const SquareRegs& q, int p, bool done, uint32_t pk[2]) {
  const int lane = lane_here();
  const Set100 empty = empty_set(q);
  const Set100 target = s_or(empty, occupied(q, 1 - p));
  // bit x of each: the neighbour of x in that direction is a target square
  const Set100 dn = s_up(target), lf = s_right(target), rt = s_left(target), up = s_down(target);
  bool scout = false;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = p_type(q.w0[h]);
    const bool mine = !done && owned_by(q.id[h], p) && movable_type(t);
    // the lane's own bit of a wave-uniform mask (a v_cndmask on the mask)
    auto bit = [&](Set100 v, uint32_t one) {
      return __builtin_amdgcn_inverse_ballot_w64(h == 0 ? v.lo : v.hi) ? one : 0u;
    };
    pk[h] = mine ? bit(dn, 1u) + bit(lf, 1u << 4) + bit(rt, 1u << 8) + bit(up, 1u << 12) : 0u;
    scout |= mine && t == kScout;
  }
  if (ballot(scout) == 0) return;
  const Set100 empty_t = ballot100(q.tid[0] == kEmpty, q.tid[1] == kEmpty);
  const Set100 target_t = s_or(empty_t, ballot100(owned_by(q.tid[0], 1 - p), owned_by(q.tid[1], 1 - p)));
  const int l = lane_here();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (done || !owned_by(q.id[h], p) || p_type(q.w0[h]) != kScout) continue;
    const int x = l + 64 * h, r = div10(x), c = x - 10 * r;
    // the Scout's row and column as 10-bit lines, position c resp. r
    const uint32_t row_e = line10(empty, 10 * r), row_t = line10(target, 10 * r);
    const uint32_t col_e = line10(empty_t, 10 * c), col_t = line10(target_t, 10 * c);
    pk[h] = line_down(col_e, col_t, r) | line_down(row_e, row_t, c) << 4 | line_up(row_e, row_t, c) << 8 |
            line_up(col_e, col_t, r) << 12;
  }
}

// The k-th destination, in ascending order, of the piece on square x whose
// counts are pk.
__device__ __forceinline__ int kth_dest(int x, uint32_t pk, int k) {
  const int nd = pk & 15u, nl = (pk >> 4) & 15u, nr = (pk >> 8) & 15u;
  if (k < nd) return x - 10 * (nd - k);
  k -= nd;
  if (k < nl) return x - (nl - k);
  k -= nl;
  if (k < nr) return x + 1 + k;
  return x + 10 * (1 + k - nr);
}

__device__ __forceinline__ int total_count(const uint32_t pk[2]) {
  return __builtin_amdgcn_readlane(dpp_incl_scan(count_of(pk[0]) + count_of(pk[1])), 63);
}

// Uniform legal action (as sample_from_words: the r-th legal action in
// ascending action order) from the counts.
// draw() gives the Philox block of the move counter, and is called only when
// there is a legal move.
template <class Draw>
__device__ __forceinline__ int sample_counts(const uint32_t pk[2], int n, Draw draw) {
  if (n <= 0) return -1;
  const uint4 u = draw();
  int r = (int)mulshift(u.x, (uint32_t)n);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = count_of(pk[h]);
    const int incl = dpp_incl_scan(c);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    if (r < total) {
      const int L = __ffsll((unsigned long long)ballot(incl > r)) - 1;
      const int k = r - (__builtin_amdgcn_readlane(incl, L) - __builtin_amdgcn_readlane(c, L));
      const int x = 64 * h + L;
      return 100 * x + kth_dest(x, (uint32_t)__builtin_amdgcn_readlane((int)pk[h], L), k);
    }
    r -= total;
  }
  return -1;
}

// Magnet policy sample (as sample_magnet) from the counts.
template <class Draw>
__device__ __forceinline__ int magnet_counts(const uint32_t pk[2], Draw draw) {
  const uint64_t has0 = ballot(pk[0] != 0), has1 = ballot(pk[1] != 0);
  const int c0 = __popcll(has0), P = c0 + __popcll(has1);
  if (P == 0) return -1;
  const uint4 u = draw();
  const int r1 = (int)mulshift(u.y, (uint32_t)P);
  const int x = r1 < c0 ? select_bit(has0, r1) : 64 + select_bit(has1, r1 - c0);
  const uint32_t pkx = (uint32_t)__builtin_amdgcn_readlane((int)(x < 64 ? pk[0] : pk[1]), x & 63);
  const int r2 = (int)mulshift(u.z, (uint32_t)count_of(pkx));
  return 100 * x + kth_dest(x, pkx, r2);
}

__device__ __forceinline__ int count_dests(const uint64_t d[4]) {
  const int c = __popcll(d[0]) + __popcll(d[1]) + __popcll(d[2]) + __popcll(d[3]);
  return __builtin_amdgcn_readlane(dpp_incl_scan(c), 63);
}

// Uniform legal action (as sample_from_words: the r-th legal action in
// ascending action order, r = bounded(x, n) of the move counter) from the
// destination sets: squares in ascending order, then destinations.
template <class Draw>
__device__ __forceinline__ int sample_dests(const uint64_t d[4], int n, Draw draw) {
  if (n <= 0) return -1;
  const uint4 u = draw();
  int r = (int)mulshift(u.x, (uint32_t)n);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = __popcll(d[2 * h]) + __popcll(d[2 * h + 1]);
    const int incl = dpp_incl_scan(c);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    if (r < total) {
      const int L = __ffsll((unsigned long long)ballot(incl > r)) - 1;
      const int k = r - __shfl(incl - c, L, 64);
      const uint64_t lo = __shfl(d[2 * h], L, 64), hi = __shfl(d[2 * h + 1], L, 64);
      const int nlo = __popcll(lo);
      const int to = k < nlo ? select_bit(lo, k) : 64 + select_bit(hi, k - nlo);
      return 100 * (64 * h + L) + to;
    }
    r -= total;
  }
  return -1;
}

// Mask words from the destination sets, parked in ts (LDS) as
// legal_mask_words parks them.
__device__ __forceinline__ void words_from_dests(const uint64_t d[4], uint64_t* ts, uint64_t w[3]) {
  const int lane = lane_here();
  ts[2 * lane] = d[0];
  ts[2 * lane + 1] = d[1];
  if (lane + 64 < kSquares) {
    ts[2 * (lane + 64)] = d[2];
    ts[2 * (lane + 64) + 1] = d[3];
  }
  if (lane == 0) { ts[200] = 0; ts[201] = 0; }
  wave_sync();
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int word = lane + 64 * g;
    uint64_t v = 0;
    if (word < kMaskWords) {
      const int a0 = 64 * word;
      const int f0 = a0 / 100;
      const int off = a0 - 100 * f0;
      const uint64_t lo = ts[2 * f0], hi = ts[2 * f0 + 1];
      v = off == 0 ? lo : off < 64 ? (lo >> off) | (hi << (64 - off)) : hi >> (off - 64);
      const int rem = 100 - off;
      if (rem < 64) v |= ts[2 * (f0 + 1)] << rem;
    }
    w[g] = v;
  }
}

// Player p has a legal move (no competitive-play rule): a movable piece next
// to an empty or enemy square.
__device__ __forceinline__ bool fast_has_move(const SquareRegs& q, int p) {
  const Set100 target = s_or(empty_set(q), occupied(q, 1 - p));
  const Set100 mov = ballot100(owned_by(q.id[0], p) && movable_type(p_type(q.w0[0])),
                               owned_by(q.id[1], p) && movable_type(p_type(q.w0[1])));
  return s_any(s_and(mov, s_nbrs(target)));
}

// apply_action for the fast path, from the registers of the pre-move state:
// the same history features, battle, death records, ring and counters, and
// the terminal check, written to the record.  The registers are left holding
// the post-move squares.  Returns done/outcome/reason.
struct FastOut {
  int done, outcome, reason;
};

__device__ __forceinline__ FastOut fast_apply(uint8_t* R, Rules rules, int action, SquareRegs& q) {
  const int lane = lane_here();
  action = __builtin_amdgcn_readfirstlane(action);
  const int from = action / 100, to = action - 100 * (action / 100);
  const int ply = __builtin_amdgcn_readfirstlane((int)hdr_u32(R, kOffPly));
  const int battleless = __builtin_amdgcn_readfirstlane((int)hdr_u32(R, kOffBattleless));
  const int ring_count = __builtin_amdgcn_readfirstlane((int)R[kOffRingCount]);
  const int pt = __builtin_amdgcn_readfirstlane((int)R[kOffRing + 2 * ((ply - 1) & 31) + 1]);
  const int p = ply & 1, o = 1 - p;
  const int X = reg_at(q.id, from);
  uint32_t wX = reg_at(q.w0, from);
  const int T = reg_at(q.id, to);
  uint32_t wT = T >= 0 ? reg_at(q.w0, to) : 0u;

  // previous move: its mover A (the opponent's piece still on its destination a)
  int A = -1, a = -1;
  bool prev_threat = false;
  if (ring_count > 0 && owned_by(reg_at(q.id, pt), o)) {
    A = reg_at(q.id, pt);
    a = pt;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int y = neighbour(a, k);
      if (y >= 0 && owned_by(reg_at(q.id, y), p)) prev_threat = true;
    }
  }

  // 1. active adjacency (pre-move): own movable pieces next to opponent
  //    pieces, except the attack being made.  Each square's opponent slot
  //    bit (1 << slot10, 0 without such a piece) is packed with the other
  //    half's into one register (square lane in bits 0-15, square 64 + lane
  //    in bits 16-31), so one lane permute fetches a neighbour of either half.
  {
    uint32_t ebit[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int sl = slot10(q.w0[h]);
      ebit[h] = owned_by(q.id[h], o) && sl >= 0 ? 1u << (sl & 15) : 0u;
    }
    const int packed = (int)(ebit[0] | ebit[1] << 16);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int x = lane + 64 * h;
      uint32_t bits = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int y = x < kSquares ? neighbour(x, k) : -1;
        const uint32_t g = (uint32_t)__shfl(packed, y & 63, 64);
        const uint32_t v = (y >= 64 ? g >> 16 : g) & 0x7FFu;
        bits |= y >= 0 && !(x == from && y == to) ? v : 0u;
      }
      if (bits && owned_by(q.id[h], p) && movable_type(p_type(q.w0[h])))
        atomicOr(&piece_words(R, q.id[h])[2], bits);
    }
  }

  // 2-4. evasion, move or battle with reveals and death records
  const bool battle = T >= 0;
  uint32_t evade = 0;
  if (A >= 0 && adjacent(from, a) && !battle && !adjacent(to, a)) {
    const int sl = slot10(reg_at(q.w0, a));
    if (sl >= 0) evade = (1u << sl) << 11;
  }
  int flag_winner = -1;
  bool attacker_alive = true;
  int res = 0;   // 0 attacker wins (or no battle), 1 defender wins, 2 tie (Table "pieces")
  if (battle) {
    const int ta = p_type(wX), td = p_type(wT);
    const bool rY = p_revealed(wT);
    if (td == kFlag) res = 0;
    else if (td == kBomb) res = ta == kMiner ? 0 : 1;
    else if (ta == kSpy && td == kMarshal) res = 0;
    else res = ta > td ? 0 : ta < td ? 1 : 2;
    wX |= 1u << 5;
    wT |= 1u << 5;
    if (td == kFlag) flag_winner = p;
    const uint32_t clear = (1u << 4) | (7u << 7) | (127u << 10);
    if (res == 0) {
      wT = (wT & ~clear) | ((rY ? 4u : 6u) << 7) | ((uint32_t)to << 10);
    } else if (res == 1) {
      attacker_alive = false;
      wX = (wX & ~clear) | ((rY ? 1u : 3u) << 7) | ((uint32_t)to << 10);
    } else {
      attacker_alive = false;
      wX = (wX & ~clear) | ((rY ? 2u : 3u) << 7) | ((uint32_t)to << 10);
      wT = (wT & ~clear) | ((rY ? 5u : 6u) << 7) | ((uint32_t)to << 10);
    }
  }
  wX |= 1u << 6;                                   // moved
  if (!adjacent(from, to)) wX |= 1u << 30;         // a long move: a known Scout
  // 5. threats by the mover from its destination (the neighbours' words are
  //    untouched by this move; `from`, now empty, held the mover)
  uint32_t threat = 0;
  if (attacker_alive) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int y = neighbour(to, k);
      if (y < 0 || !owned_by(reg_at(q.id, y), o)) continue;
      const int sl = slot10(reg_at(q.w0, y));
      if (sl >= 0) threat |= 1u << sl;
    }
  }
  // 6. protection: a non-battle reply to a threat that newly puts the mover
  //    next to a square beside the threatener (the squares looked at are
  //    neither `from` nor `to`, so their registers are current)
  uint32_t prot2 = 0, prot3 = 0;
  if (!battle && A >= 0 && prev_threat) {
    const uint32_t bitA = 1u << slot13(reg_at(q.w0, a));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int sq = neighbour(a, k);
      if (sq < 0 || is_lake_sq(sq)) continue;
      if (!adjacent(sq, to) || sq == from || adjacent(sq, from)) continue;
      const int oid = reg_at(q.id, sq);
      if (owned_by(oid, p)) {
        prot2 |= (1u << slot13(reg_at(q.w0, sq))) << 11;
        prot3 |= bitA;
        if (lane == 0) {
          uint32_t* pb = piece_words(R, oid);
          atomicOr(&pb[3], (1u << slot13(wX)) << 13);
          atomicOr(&pb[0], bitA << 17);
        }
      } else if (oid == kEmpty) {
        prot2 |= (1u << 11) << 11;
        prot3 |= bitA;
      }
    }
  }
  // 7-8. record writes: board, pieces, ring and counters
  const int to_id = !battle || res == 0 ? X : res == 2 ? kEmpty : T;
  if (lane == 0) {
    uint32_t* px = piece_words(R, X);
    set_board(R, from, kEmpty);
    set_board(R, to, to_id);
    px[0] = wX;
    if (battle) piece_words(R, T)[0] = wT;
    if (evade | threat) atomicOr(&px[1], evade | threat);
    if (prot2) atomicOr(&px[2], prot2);
    if (prot3) atomicOr(&px[3], prot3);
    const int slot = ply & 31;
    R[kOffRing + 2 * slot] = (uint8_t)from;
    R[kOffRing + 2 * slot + 1] = (uint8_t)to;
    if (ring_count < 32) R[kOffRingCount] = (uint8_t)(ring_count + 1);
    set_hdr_u32(R, kOffPly, (uint32_t)(ply + 1));
    set_hdr_u32(R, kOffBattleless, battle ? 0u : (uint32_t)(battleless + 1));
  }
  // the registers of the two squares the move changed, then the terminal
  // check (App. A; App. D.1)
  const uint32_t to_w0 = to_id == X ? wX : to_id == T ? wT : 0u;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int x = lane + 64 * h;
    if (x == from) { q.id[h] = kEmpty; q.w0[h] = 0u; }
    if (x == to) { q.id[h] = to_id; q.w0[h] = to_w0; }
  }
  FastOut out{0, 0, kReasonNone};
  if (flag_winner >= 0) {
    out = FastOut{1, flag_winner == 0 ? 1 : -1, kReasonFlag};
  } else if (!fast_has_move(q, o)) {
    out = fast_has_move(q, p) ? FastOut{1, p == 0 ? 1 : -1, kReasonForcedWin} : FastOut{1, 0, kReasonForcedDraw};
  } else if ((battle ? 0 : battleless + 1) >= rules.k_battleless) {
    out = FastOut{1, 0, kReasonKMove};
  } else if (ply + 1 >= rules.max_moves) {
    out = FastOut{1, 0, kReasonMaxMoves};
  }
  if (lane == 0) {
    R[kOffDone] = (uint8_t)out.done;
    R[kOffOutcome] = (uint8_t)(int8_t)out.outcome;
    R[kOffReason] = (uint8_t)out.reason;
  }
  return out;
}

// reset_game for the fast path: a fresh setup is terminal only when a player
// to move has no movable piece with room, checked on the registers.
__device__ __forceinline__ void fast_reset_game(uint8_t* R, uint8_t* scratch, Rules rules, uint32_t game_id,
                                                uint32_t episode, uint32_t redraws) {
  for (int guard = 0;; ++guard) {
    fresh_setup(R, scratch, rules.seed, game_id, episode, redraws);
    SquareRegs q;
    load_regs(R, q);
    FastOut t{0, 0, kReasonNone};
    if (!fast_has_move(q, 0)) t = fast_has_move(q, 1) ? FastOut{1, -1, kReasonForcedWin} : FastOut{1, 0, kReasonForcedDraw};
    if (lane_id() == 0) {
      R[kOffDone] = (uint8_t)t.done;
      R[kOffOutcome] = (uint8_t)(int8_t)t.outcome;
      R[kOffReason] = (uint8_t)t.reason;
    }
    wave_sync();
    // a setup that is already terminal is replaced by the next episode's
    // (probability ~4e-6 per game); the bound only guards against a hang
    if (!(t.done && rules.auto_reset && guard < 1000)) break;
    ++episode;
    ++redraws;
  }
}

// step_game for the fast path (drawn actions, no competitive-play rule).
__device__ __forceinline__ StepOut fast_step_game(uint8_t* R, uint8_t* scratch, uint8_t* work, Rules rules,
                                                  int action, SquareRegs& q) {
  StepOut o{0, 0, 0, 0, false};
  if (!R[kOffDone]) {
    if (action == -1) return o;
    const FastOut f = fast_apply(R, rules, action, q);
    if (!f.done) return o;
    wave_sync();
  }
  o.done = 1;
  o.outcome = (int8_t)R[kOffOutcome];
  o.reason = R[kOffReason];
  o.ep_len = (int)hdr_u32(R, kOffPly);
  (void)work;
  if (rules.auto_reset)
    fast_reset_game(R, scratch, rules, hdr_u32(R, kOffGameId), hdr_u32(R, kOffEpisode) + 1,
                    hdr_u32(R, kOffRedraws));
  return o;
}

// ---------------------------------------------------------------- probabilities
// Channels 12-35 (App. C.1): chance that a piece of unknown type has type T
// when the unknown types are a uniform assignment of the owner's remaining
// multiset in which no moved piece is a Flag or Bomb.  Revealed pieces and
// known Scouts (a move of more than one square, App. A) are out of the
// multiset.  With H unknown pieces, I unknown Flag+Bomb, M moved unknown,
// U = H - M unmoved unknown and n_T remaining of T:
// moved: n_T/(H-I) for movable T, 0 otherwise; unmoved: n_T/U for Flag/Bomb,
// n_T(U-I)/(U(H-I)) for movable T.  Stored as round-half-up(255 p) in
// probq[owner][moved][type].
__device__ __forceinline__ uint32_t quant255(uint32_t num, uint32_t den) {
  return den == 0 ? 0u : (510u * num + den) / (2u * den);
}

__device__ __forceinline__ void compute_probq(const uint8_t* R, uint8_t* slab) {
  const int lane = lane_id();
  int* cnt = reinterpret_cast<int*>(slab + kSlabCounts);   // known[2][12], H[2], M[2]
  if (lane < 28) cnt[lane] = 0;
  wave_sync();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int id = lane + 64 * h;
    if (id < kPieces) {
      uint32_t w0 = piece_words(R, id)[0];
      int w = owner(id);
      if (!p_alive(w0) || p_known(w0)) {
        atomicAdd(&cnt[12 * w + p_type(w0)], 1);
      } else {
        atomicAdd(&cnt[24 + w], 1);
        if (p_moved(w0)) atomicAdd(&cnt[26 + w], 1);
      }
    }
  }
  wave_sync();
  if (lane < 48) {
    const int w = lane / 24, m = (lane / 12) & 1, t = lane % 12;
    const int n_t = initial_count(t) - cnt[12 * w + t];
    const int H = cnt[24 + w], M = cnt[26 + w], U = H - M;
    const int I = (initial_count(kFlag) - cnt[12 * w + kFlag]) + (initial_count(kBomb) - cnt[12 * w + kBomb]);
    uint32_t v;
    if (m) v = movable_type(t) ? quant255((uint32_t)n_t, (uint32_t)(H - I)) : 0u;
    else if (!movable_type(t)) v = quant255((uint32_t)n_t, (uint32_t)U);
    else v = quant255((uint32_t)(n_t * (U - I)), (uint32_t)(U * (H - I)));
    slab[kSlabProbQ + lane] = (uint8_t)v;
  }
  wave_sync();
}

// ---------------------------------------------------------------- encoding
// Byte v at (channel c, frame square f) of observer o's image segment, kept
// only when c lies in [c_lo, c_hi).  Observer 1's segment follows observer 0's.
struct SegWriter {
  uint8_t* img;
  int c_lo, c_hi, seg_bytes;
  __device__ __forceinline__ void put(int o, int c, int f, uint8_t v) const {
    if (c >= c_lo && c < c_hi) img[o * seg_bytes + (c - c_lo) * 100 + f] = v;
  }
  __device__ __forceinline__ bool overlaps(int a, int b) const { return a < c_hi && b > c_lo; }
};

__device__ __forceinline__ int frame_of(int o, int s) { return o == 0 ? s : 99 - s; }

// Scatter the non-zero bytes of both observers' channels [c_lo, c_hi) into the
// zeroed image segments (App. C.1 channel table, App. C.2 move planes).  Every
// attribute of a piece appears twice: in its owner's "own" channel and in the
// opponent's "opponent" channel, each in that observer's frame.
__device__ __forceinline__ void scatter_segment(const uint8_t* R, const uint8_t* slab, Rules rules,
                                const SegWriter& W) {
  const int lane = lane_id();
  const int ply = (int)hdr_u32(R, kOffPly);
  // 41-42: fractions of the move budget and of the k-move budget, on every square
  if (W.overlaps(41, 43)) {
    const uint8_t v41 = (uint8_t)quant255((uint32_t)ply, (uint32_t)rules.max_moves);
    const uint8_t v42 = (uint8_t)quant255(hdr_u32(R, kOffBattleless), (uint32_t)rules.k_battleless);
    for (int f = lane; f < kSquares; f += 64) {
      W.put(0, 41, f, v41);
      W.put(0, 42, f, v42);
      W.put(1, 41, f, v41);
      W.put(1, 42, f, v42);
    }
  }
  // squares
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    const int s = lane + 64 * h;
    if (s >= kSquares) break;
    const int id = board_at(R, s);
    if (id == kLake) continue;
    if (id == kEmpty) {
      W.put(0, 38, s, 1);
      W.put(1, 38, 99 - s, 1);
      continue;
    }
    const int w = owner(id), e = 1 - w;      // owner and opponent observers
    const int fw = frame_of(w, s), fe = frame_of(e, s);
    const uint32_t* pw = piece_words(R, id);
    const uint32_t w0 = pw[0];
    const int t = p_type(w0);
    const bool rev = p_revealed(w0), mv = p_moved(w0);
    if (W.overlaps(0, 41)) {
      W.put(w, t, fw, 1);                                  // 0-11 own type
      if (!rev) { W.put(w, 36, fw, 1); W.put(e, 37, fe, 1); }
      if (mv) { W.put(w, 39, fw, 1); W.put(e, 40, fe, 1); }
      if (p_known(w0)) {                                   // 12-35 known type
        W.put(w, 24 + t, fw, 255);
        W.put(e, 12 + t, fe, 255);
      } else {                                             // 12-35 probabilities
        const uint8_t* pq = slab + kSlabProbQ + 24 * w + 12 * (mv ? 1 : 0);
        for (int k = 0; k < 12; ++k) {
          const uint8_t v = pq[k];
          if (v) { W.put(w, 24 + k, fw, v); W.put(e, 12 + k, fe, v); }
        }
      }
    }
    if (W.overlaps(43, 109)) {                             // threat, evade, adjacency
      uint32_t th = pw[1] & 0x7FFu, ev = (pw[1] >> 11) & 0x7FFu, ad = pw[2] & 0x7FFu;
      while (th) { int j = __ffs(th) - 1; th &= th - 1; W.put(w, 43 + j, fw, 1); W.put(e, 76 + j, fe, 1); }
      while (ev) { int j = __ffs(ev) - 1; ev &= ev - 1; W.put(w, 54 + j, fw, 1); W.put(e, 87 + j, fe, 1); }
      while (ad) { int j = __ffs(ad) - 1; ad &= ad - 1; W.put(w, 65 + j, fw, 1); W.put(e, 98 + j, fe, 1); }
    }
    if (W.overlaps(251, 355)) {                            // protection groups
      uint32_t pr = (pw[2] >> 11) & 0x1FFFu, pa = pw[3] & 0x1FFFu;
      uint32_t bb = (pw[3] >> 13) & 0x1FFFu, ba = (w0 >> 17) & 0x1FFFu;
      while (pr) { int j = __ffs(pr) - 1; pr &= pr - 1; W.put(w, 251 + j, fw, 1); W.put(e, 303 + j, fe, 1); }
      while (pa) { int j = __ffs(pa) - 1; pa &= pa - 1; W.put(w, 264 + j, fw, 1); W.put(e, 316 + j, fe, 1); }
      while (bb) { int j = __ffs(bb) - 1; bb &= bb - 1; W.put(w, 277 + j, fw, 1); W.put(e, 329 + j, fe, 1); }
      while (ba) { int j = __ffs(ba) - 1; ba &= ba - 1; W.put(w, 290 + j, fw, 1); W.put(e, 342 + j, fe, 1); }
    }
    if (W.overlaps(355, 455)) {                            // start square of this piece
      const int st = start_sq(id);
      W.put(w, 355 + frame_of(w, st), fw, 1);
      W.put(e, 355 + frame_of(e, st), fe, 1);
    }
  }
  // captured pieces: start squares (109-130) and death square x cause (131-250)
  if (W.overlaps(109, 251)) {
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      const int id = lane + 64 * h;
      if (id >= kPieces) break;
      const uint32_t w0 = piece_words(R, id)[0];
      if (p_alive(w0)) continue;
      const int t = p_type(w0);
      if (t == kFlag) continue;
      const int w = owner(id), e = 1 - w;
      const int st = start_sq(id), slot = t == kBomb ? 10 : t;
      W.put(w, 109 + slot, frame_of(w, st), 1);
      W.put(e, 120 + slot, frame_of(e, st), 1);
      if (t <= kMarshal) {
        const int cause = (w0 >> 7) & 7, dsq = (w0 >> 10) & 127;
        W.put(w, 131 + 10 * (cause - 1) + t, frame_of(w, dsq), 1);
        W.put(e, 191 + 10 * (cause - 1) + t, frame_of(e, dsq), 1);
      }
    }
  }
  // recent moves (456-487), most recent first
  if (W.overlaps(456, 488)) {
    const int rc = R[kOffRingCount];
    if (lane < rc) {
      const int slot = (ply - 1 - lane) & 31;
      const int fr = R[kOffRing + 2 * slot], to = R[kOffRing + 2 * slot + 1];
      W.put(0, 456 + lane, to, 0x01);
      W.put(0, 456 + lane, fr, 0xFF);
      W.put(1, 456 + lane, 99 - to, 0x01);
      W.put(1, 456 + lane, 99 - fr, 0xFF);
    }
  }
}

// The LDS image region of a wave's slab is kept all-zero between uses: it is
// cleared once when a kernel starts, every segment's copy-out clears what it
// read, and the legal-move phase clears the destination sets it parked there.
__device__ __forceinline__ void clear_lds(uint8_t* p, int bytes) {
  u32x4* q = reinterpret_cast<u32x4*>(p);
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (int k = lane_id(); k < bytes / 16; k += 64) q[k] = z;
  wave_sync();
}

// Bytes of the 101 destination sets legal_mask_words parks in the image.
constexpr int kDestSetBytes = 101 * 16;

// Stream `chunks` 16-byte chunks of an LDS image to global memory, four loads
// in flight per lane, clearing behind.  Plain stores: on gfx950 the
// non-temporal hint measured slower for this write stream.
__device__ __forceinline__ void stream_out(u32x4* im, u32x4* dst, int chunks) {
  const u32x4 z = {0u, 0u, 0u, 0u};
  int k = lane_id();
  for (; k + 192 < chunks; k += 256) {
    u32x4 v0 = im[k], v1 = im[k + 64], v2 = im[k + 128], v3 = im[k + 192];
    im[k] = z;
    im[k + 64] = z;
    im[k + 128] = z;
    im[k + 192] = z;
    *(dst + k) = v0;
    *(dst + k + 64) = v1;
    *(dst + k + 128) = v2;
    *(dst + k + 192) = v3;
  }
  for (; k < chunks; k += 64) {
    u32x4 v = im[k];
    im[k] = z;
    *(dst + k) = v;
  }
}

// Encode both observers of the game staged in R into obs (global, 97600
// bytes) with the byte-image layout: per segment of channels, scatter both
// observers' non-zero bytes into the zero LDS images, then stream both
// segments to HBM.
__device__ __forceinline__ void encode_game_bytes(const uint8_t* R, uint8_t* slab, Rules rules, int segments,
                                  uint8_t* obs) {
  const int segc = seg_channels_for(segments), segb = seg_bytes_for(segments);
  uint8_t* img = slab + kSlabImage;
#pragma unroll 1
  for (int c_lo = 0; c_lo < kChannels; c_lo += segc) {
    const int c_hi = c_lo + segc < kChannels ? c_lo + segc : kChannels;
    const int chunks = (c_hi - c_lo) * 100 / 16;
    SegWriter W{img, c_lo, c_hi, segb};
    scatter_segment(R, slab, rules, W);
    wave_sync();
    // both observers' images, or the acting player's only
    const int first = rules.acting_obs ? (int)(hdr_u32(R, kOffPly) & 1) : 0;
    const int count = rules.acting_obs ? 1 : 2;
#pragma unroll 1
    for (int k = 0; k < count; ++k)
      stream_out(reinterpret_cast<u32x4*>(img + (first + k) * segb),
                 reinterpret_cast<u32x4*>(obs + k * kObsPerObserver + c_lo * 100), chunks);
    // the image must be left zero: clear the other observer's, not streamed
    if (rules.acting_obs) clear_lds(img + (1 - first) * segb, 16 * chunks);
    wave_sync();
  }
}

// ---------------------------------------------------------------- bit planes
__device__ __forceinline__ void plane_set(uint8_t* slab, int o, int c, int f) {
  const int bit = 100 * c + f;
  uint32_t* bm = reinterpret_cast<uint32_t*>(slab + (o ? kBitsPlane1 : kBitsPlane0));
  atomicOr(&bm[bit >> 5], 1u << (bit & 31));
}

// 4 bits -> 4 bytes holding 0 or 1
__device__ __forceinline__ uint32_t expand4(uint32_t n) { return (n * 0x00204081u) & 0x01010101u; }

// Build both observers' bit planes, probability categories and tables in one
// pass over squares, dead pieces and the move ring (App. C.1, C.2).  Planes
// must be zero on entry.  Probability channels 12-35 take their hidden-piece
// values from per-square categories (1/2 opponent hidden moved/unmoved, 3/4
// own hidden moved/unmoved) and a per-channel table; the planes carry only the
// 255 of revealed types there.
__device__ __forceinline__ void build_bitplanes(const uint8_t* R, uint8_t* slab) {
  const int lane = lane_id();
  const int ply = (int)hdr_u32(R, kOffPly);
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    const int s = lane + 64 * h;
    if (s >= kSquares) break;
    const int id = board_at(R, s);
    uint8_t cat0 = 0, cat1 = 0;
    if (id == kEmpty) {
      plane_set(slab, 0, 38, s);
      plane_set(slab, 1, 38, 99 - s);
    } else if (id >= 0) {
      const int w = owner(id), e = 1 - w;
      const int fw = frame_of(w, s), fe = frame_of(e, s);
      const uint32_t* pw = piece_words(R, id);
      const uint32_t w0 = pw[0];
      const int t = p_type(w0);
      const bool rev = p_revealed(w0), mv = p_moved(w0);
      plane_set(slab, w, t, fw);
      if (!rev) {
        plane_set(slab, w, 36, fw);
        plane_set(slab, e, 37, fe);
      }
      if (p_known(w0)) {
        plane_set(slab, w, 24 + t, fw);
        plane_set(slab, e, 12 + t, fe);
      } else {
        const uint8_t own_cat = mv ? 3 : 4, opp_cat = mv ? 1 : 2;
        if (w == 0) { cat0 = own_cat; cat1 = opp_cat; } else { cat1 = own_cat; cat0 = opp_cat; }
      }
      if (mv) {
        plane_set(slab, w, 39, fw);
        plane_set(slab, e, 40, fe);
      }
      uint32_t th = pw[1] & 0x7FFu, ev = (pw[1] >> 11) & 0x7FFu, ad = pw[2] & 0x7FFu;
      while (th) { int j = __ffs(th) - 1; th &= th - 1; plane_set(slab, w, 43 + j, fw); plane_set(slab, e, 76 + j, fe); }
      while (ev) { int j = __ffs(ev) - 1; ev &= ev - 1; plane_set(slab, w, 54 + j, fw); plane_set(slab, e, 87 + j, fe); }
      while (ad) { int j = __ffs(ad) - 1; ad &= ad - 1; plane_set(slab, w, 65 + j, fw); plane_set(slab, e, 98 + j, fe); }
      uint32_t pr = (pw[2] >> 11) & 0x1FFFu, pa = pw[3] & 0x1FFFu;
      uint32_t bb = (pw[3] >> 13) & 0x1FFFu, ba = (w0 >> 17) & 0x1FFFu;
      while (pr) { int j = __ffs(pr) - 1; pr &= pr - 1; plane_set(slab, w, 251 + j, fw); plane_set(slab, e, 303 + j, fe); }
      while (pa) { int j = __ffs(pa) - 1; pa &= pa - 1; plane_set(slab, w, 264 + j, fw); plane_set(slab, e, 316 + j, fe); }
      while (bb) { int j = __ffs(bb) - 1; bb &= bb - 1; plane_set(slab, w, 277 + j, fw); plane_set(slab, e, 329 + j, fe); }
      while (ba) { int j = __ffs(ba) - 1; ba &= ba - 1; plane_set(slab, w, 290 + j, fw); plane_set(slab, e, 342 + j, fe); }
      const int st = start_sq(id);
      plane_set(slab, w, 355 + frame_of(w, st), fw);
      plane_set(slab, e, 355 + frame_of(e, st), fe);
    }
    slab[kBitsCat0 + s] = cat0;
    slab[kBitsCat1 + 99 - s] = cat1;
  }
  // captured pieces: start squares (109-130) and death square x cause (131-250)
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    const int id = lane + 64 * h;
    if (id >= kPieces) break;
    const uint32_t w0 = piece_words(R, id)[0];
    if (p_alive(w0)) continue;
    const int t = p_type(w0);
    if (t == kFlag) continue;
    const int w = owner(id), e = 1 - w;
    const int st = start_sq(id), slot = t == kBomb ? 10 : t;
    plane_set(slab, w, 109 + slot, frame_of(w, st));
    plane_set(slab, e, 120 + slot, frame_of(e, st));
    if (t <= kMarshal) {
      const int cause = (w0 >> 7) & 7, dsq = (w0 >> 10) & 127;
      plane_set(slab, w, 131 + 10 * (cause - 1) + t, frame_of(w, dsq));
      plane_set(slab, e, 191 + 10 * (cause - 1) + t, frame_of(e, dsq));
    }
  }
  // recent moves (456-487): destinations in the planes, sources in the side planes
  const int rc = R[kOffRingCount];
  if (lane < rc) {
    const int slot = (ply - 1 - lane) & 31;
    const int fr = R[kOffRing + 2 * slot], to = R[kOffRing + 2 * slot + 1];
    plane_set(slab, 0, 456 + lane, to);
    plane_set(slab, 1, 456 + lane, 99 - to);
    uint32_t* m0 = reinterpret_cast<uint32_t*>(slab + kBitsMove0);
    uint32_t* m1 = reinterpret_cast<uint32_t*>(slab + kBitsMove1);
    const int b0 = 100 * lane + fr, b1 = 100 * lane + 99 - fr;
    atomicOr(&m0[b0 >> 5], 1u << (b0 & 31));
    atomicOr(&m1[b1 >> 5], 1u << (b1 & 31));
  }
  // probability tables: entry c-12 of observer o, indexed by category
  if (lane < 48) {
    const int o = lane / 24, j = lane % 24;
    const uint8_t* pq = slab + kSlabProbQ;
    uint64_t tab;
    if (j < 12) {   // channel 12 + j: the opponent's pieces, type j
      const int z = 1 - o;
      tab = ((uint64_t)pq[24 * z + 12 + j] << 8) | ((uint64_t)pq[24 * z + j] << 16);
    } else {        // channel 24 + (j - 12): own pieces, type j - 12
      tab = ((uint64_t)pq[24 * o + 12 + (j - 12)] << 24) | ((uint64_t)pq[24 * o + (j - 12)] << 32);
    }
    reinterpret_cast<uint64_t*>(slab + kBitsTab)[lane] = tab;
  }
  wave_sync();
}

// Expand observer o's bit planes to 48800 bytes in global memory: each lane
// turns 16 plane bits into one 16-byte chunk; consecutive lanes write
// consecutive chunks (1 KB per wave store).
template <int L>
__device__ __forceinline__ void stream_planes(const uint8_t* slab, int o, uint32_t c41, uint32_t c42, uint8_t* out) {
  // layout 1 keeps both observers' planes side by side; layout 7 one set
  const uint16_t* bm = reinterpret_cast<const uint16_t*>(slab + (L == kLayoutBits ? kBitsPlane0 + o * kBitsPlane : kB1Plane));
  const uint16_t* mv =
      reinterpret_cast<const uint16_t*>(slab + (L == kLayoutBits ? kBitsMove0 + o * kBitsMovePlane : kB1Move));
  const uint8_t* cat = slab + (L == kLayoutBits ? kBitsCat0 + o * 112 : kB1Cat);
  const uint64_t* tab = reinterpret_cast<const uint64_t*>(slab + (L == kLayoutBits ? kBitsTab + o * 192 : kB1Tab));
  u32x4* dst = reinterpret_cast<u32x4*>(out);
  constexpr int kChunks = kObsPerObserver / 16;   // 3050
#pragma unroll 2
  for (int k = lane_id(); k < kChunks; k += 64) {
    const uint32_t x = bm[k];
    uint32_t d[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) d[j] = expand4((x >> (4 * j)) & 15u);
    if (k >= 75 && k < 269) {
      // channels 12-35 (probabilities, 255 for known types) and 41-42 (fractions)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int b = 16 * k + 4 * j;
        const int c = b / 100, f0 = b - 100 * c;
        if (c >= 12 && c < 36) {
          const uint32_t cats = *reinterpret_cast<const uint32_t*>(cat + f0);
          const uint64_t tb = tab[c - 12];
          d[j] = __builtin_amdgcn_perm((uint32_t)(tb >> 32), (uint32_t)tb, cats) | (d[j] * 0xFFu);
        } else if (c == 41) {
          d[j] = c41;
        } else if (c == 42) {
          d[j] = c42;
        }
      }
    } else if (k >= 2850) {
      // channels 456-487: +1 destinations from the planes, -1 (0xFF) sources
      const uint32_t y = mv[k - 2850];
#pragma unroll
      for (int j = 0; j < 4; ++j) d[j] |= expand4((y >> (4 * j)) & 15u) * 0xFFu;
    }
    const u32x4 v = {d[0], d[1], d[2], d[3]};
    *(dst + k) = v;
  }
}

__device__ __forceinline__ void stream_bitplanes(const uint8_t* slab, int o, uint32_t c41, uint32_t c42,
                                                 uint8_t* out) {
  stream_planes<kLayoutBits>(slab, o, c41, c42, out);
}

// Observer o's planes only (layout kLayoutBits1): the same channels as
// build_bitplanes, each piece seen from o's side, in o's frame.
__device__ __forceinline__ void build_bitplanes1(const uint8_t* R, uint8_t* slab, int o) {
  const int lane = lane_id();
  const int ply = (int)hdr_u32(R, kOffPly);
  uint32_t* bm = reinterpret_cast<uint32_t*>(slab + kB1Plane);
  auto set = [&](int c, int f) {
    const int bit = 100 * c + f;
    atomicOr(&bm[bit >> 5], 1u << (bit & 31));
  };
  auto fr = [&](int sq) { return o == 0 ? sq : 99 - sq; };
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    const int s = lane + 64 * h;
    if (s >= kSquares) break;
    const int id = board_at(R, s), f = fr(s);
    uint8_t cat = 0;
    if (id == kEmpty) {
      set(38, f);
    } else if (id >= 0) {
      const bool own = owner(id) == o;
      const uint32_t* pw = piece_words(R, id);
      const uint32_t w0 = pw[0];
      const int t = p_type(w0);
      const bool rev = p_revealed(w0), mv = p_moved(w0);
      if (own) set(t, f);
      if (!rev) set(own ? 36 : 37, f);
      if (p_known(w0)) set((own ? 24 : 12) + t, f);
      else cat = own ? (mv ? 3 : 4) : (mv ? 1 : 2);
      if (mv) set(own ? 39 : 40, f);
      uint32_t th = pw[1] & 0x7FFu, ev = (pw[1] >> 11) & 0x7FFu, ad = pw[2] & 0x7FFu;
      const int b_th = own ? 43 : 76, b_ev = own ? 54 : 87, b_ad = own ? 65 : 98;
      while (th) { int j = __ffs(th) - 1; th &= th - 1; set(b_th + j, f); }
      while (ev) { int j = __ffs(ev) - 1; ev &= ev - 1; set(b_ev + j, f); }
      while (ad) { int j = __ffs(ad) - 1; ad &= ad - 1; set(b_ad + j, f); }
      uint32_t pr = (pw[2] >> 11) & 0x1FFFu, pa = pw[3] & 0x1FFFu;
      uint32_t bb = (pw[3] >> 13) & 0x1FFFu, ba = (w0 >> 17) & 0x1FFFu;
      const int b_pr = own ? 251 : 303, b_pa = own ? 264 : 316, b_bb = own ? 277 : 329, b_ba = own ? 290 : 342;
      while (pr) { int j = __ffs(pr) - 1; pr &= pr - 1; set(b_pr + j, f); }
      while (pa) { int j = __ffs(pa) - 1; pa &= pa - 1; set(b_pa + j, f); }
      while (bb) { int j = __ffs(bb) - 1; bb &= bb - 1; set(b_bb + j, f); }
      while (ba) { int j = __ffs(ba) - 1; ba &= ba - 1; set(b_ba + j, f); }
      set(355 + fr(start_sq(id)), f);
    }
    slab[kB1Cat + f] = cat;
  }
  // captured pieces: start squares (109-130) and death square x cause (131-250)
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    const int id = lane + 64 * h;
    if (id >= kPieces) break;
    const uint32_t w0 = piece_words(R, id)[0];
    if (p_alive(w0)) continue;
    const int t = p_type(w0);
    if (t == kFlag) continue;
    const bool own = owner(id) == o;
    const int slot = t == kBomb ? 10 : t;
    set((own ? 109 : 120) + slot, fr(start_sq(id)));
    if (t <= kMarshal) {
      const int cause = (w0 >> 7) & 7, dsq = (w0 >> 10) & 127;
      set((own ? 131 : 191) + 10 * (cause - 1) + t, fr(dsq));
    }
  }
  // recent moves (456-487): destinations in the plane, sources in the side plane
  const int rc = R[kOffRingCount];
  if (lane < rc) {
    const int slot = (ply - 1 - lane) & 31;
    const int from = R[kOffRing + 2 * slot], to = R[kOffRing + 2 * slot + 1];
    set(456 + lane, fr(to));
    uint32_t* m = reinterpret_cast<uint32_t*>(slab + kB1Move);
    const int b = 100 * lane + fr(from);
    atomicOr(&m[b >> 5], 1u << (b & 31));
  }
  // probability table of observer o, indexed by category
  if (lane < 24) {
    const int j = lane;
    const uint8_t* pq = slab + kSlabProbQ;
    uint64_t tab;
    if (j < 12) {   // channel 12 + j: the opponent's pieces, type j
      const int z = 1 - o;
      tab = ((uint64_t)pq[24 * z + 12 + j] << 8) | ((uint64_t)pq[24 * z + j] << 16);
    } else {        // channel 24 + (j - 12): own pieces, type j - 12
      tab = ((uint64_t)pq[24 * o + 12 + (j - 12)] << 24) | ((uint64_t)pq[24 * o + (j - 12)] << 32);
    }
    reinterpret_cast<uint64_t*>(slab + kB1Tab)[j] = tab;
  }
  wave_sync();
}

// Layout kLayoutBits1: build, stream and clear one observer's planes at a time.
__device__ __forceinline__ void encode_game_bits1(const uint8_t* R, uint8_t* slab, Rules rules, uint8_t* obs) {
  const uint32_t c41 = 0x01010101u * quant255(hdr_u32(R, kOffPly), (uint32_t)rules.max_moves);
  const uint32_t c42 = 0x01010101u * quant255(hdr_u32(R, kOffBattleless), (uint32_t)rules.k_battleless);
  const int first = rules.acting_obs ? (int)(hdr_u32(R, kOffPly) & 1) : 0;
  const int count = rules.acting_obs ? 1 : 2;
#pragma unroll 1
  for (int k = 0; k < count; ++k) {
    clear_lds(slab + kSlabImage, image_bytes_for(kLayoutBits1));
    build_bitplanes1(R, slab, first + k);
    stream_planes<kLayoutBits1>(slab, 0, c41, c42, obs + k * kObsPerObserver);
    wave_sync();
  }
}

__device__ __forceinline__ void encode_game_bits(const uint8_t* R, uint8_t* slab, Rules rules, uint8_t* obs) {
  clear_lds(slab + kSlabImage, image_bytes_for(kLayoutBits));
  build_bitplanes(R, slab);
  const uint32_t c41 = 0x01010101u * quant255(hdr_u32(R, kOffPly), (uint32_t)rules.max_moves);
  const uint32_t c42 = 0x01010101u * quant255(hdr_u32(R, kOffBattleless), (uint32_t)rules.k_battleless);
  // both observers, or the acting player's planes only
  const int first = rules.acting_obs ? (int)(hdr_u32(R, kOffPly) & 1) : 0;
  const int count = rules.acting_obs ? 1 : 2;
#pragma unroll 1
  for (int k = 0; k < count; ++k) stream_bitplanes(slab, first + k, c41, c42, obs + k * kObsPerObserver);
  wave_sync();
}

// Encode both observers with the given LDS layout.  The byte-image layouts
// expect a zero image on entry and leave it zero; the bit-plane layout clears
// its planes itself.
__device__ __forceinline__ void encode_game(const uint8_t* R, uint8_t* slab, Rules rules, int layout,
                            uint8_t* obs) {
  if (layout == kLayoutBits) encode_game_bits(R, slab, rules, obs);
  else if (layout == kLayoutBits1) encode_game_bits1(R, slab, rules, obs);
  else encode_game_bytes(R, slab, rules, segments_of(layout), obs);
}

// ---------------------------------------------------------------- resampling
// Hidden types of the player not to move redrawn uniformly among assignments
// consistent with public information (paper section 2.5; belief samples are
// replaced by this uniform model; revealed pieces and known Scouts keep their
// types): first the Flag and Bombs among the unmoved hidden pieces (partial Fisher-Yates in ascending id order, Flag first), then
// the movable multiset shuffled over the remaining hidden pieces in ascending
// id order.  The random words (Philox counter (new id, block, episode, 3),
// words x, y, z, w of each block in turn) are drawn one per lane, the two
// shuffles run as swaps between lanes, and the new types are patched into the
// record's 16-byte chunks as they are stored, so one source serves many
// resamples without being copied.

// Swap the values of lanes a and b (a, b wave-uniform).
__device__ __forceinline__ int lane_swap(int v, int a, int b) {
  const int va = __builtin_amdgcn_readlane(v, a), vb = __builtin_amdgcn_readlane(v, b);
  const int lane = lane_id();
  return lane == a ? vb : lane == b ? va : v;
}

// What every resample of one source shares.
struct ResampleSource {
  int z, nu, I, L, nflag;
  uint32_t episode;
  uint64_t hidden;   // bit m: piece 40 z + m is alive and of unknown type
  int unmoved;       // lane m < nu: id of the m-th unmoved hidden piece of z, ascending
  int list;          // lane m < L: the m-th type of z's hidden movable multiset, sorted
  uint4 c0, c1;      // the record's 16-byte chunks lane and 64 + lane (lane < 32)
};

__device__ __forceinline__ ResampleSource resample_prepare(const uint8_t* R) {
  const int lane = lane_id();
  ResampleSource S;
  S.z = 1 - (int)(hdr_u32(R, kOffPly) & 1);
  S.episode = hdr_u32(R, kOffEpisode);
  const bool mine = lane < 40;
  const uint32_t w0 = mine ? piece_words(R, 40 * S.z + lane)[0] : 0u;
  const bool known = mine && (!p_alive(w0) || p_known(w0));
  const bool hid = mine && p_alive(w0) && !p_known(w0);
  const int t = p_type(w0);
  S.hidden = ballot(hid);
  const uint64_t um = ballot(hid && !p_moved(w0));
  S.nu = __popcll(um);
  S.unmoved = lane < S.nu ? 40 * S.z + select_bit(um, lane) : 0;
  // hidden counts per type: the initial multiset minus the known pieces
  int acc = 0, ty = 0;
  S.L = 0;
#pragma unroll
  for (int k = 0; k <= kMarshal; ++k) {
    const int c = initial_count(k) - __popcll(ballot(known && t == k));
    acc += c;
    ty += lane >= acc ? 1 : 0;
  }
  S.L = acc;
  S.list = ty;
  S.nflag = initial_count(kFlag) - __popcll(ballot(known && t == kFlag));
  S.I = S.nflag + initial_count(kBomb) - __popcll(ballot(known && t == kBomb));
  const uint4* r4 = reinterpret_cast<const uint4*>(R);
  S.c0 = r4[lane];
  S.c1 = lane < 32 ? r4[64 + lane] : make_uint4(0, 0, 0, 0);
  return S;
}

// Resamples of one source, one per lane: lane r draws resample r with game id
// id0 + r, and the wave then stores the first cnt of them as records at
// out, out + 1536, ...  A lane keeps its own copies of the source's unmoved
// list and type list in LDS rows (um + r * kUmStride, ls + r * kLsStride,
// odd strides, so a column and a row both fall in distinct banks) and shuffles
// them with its own words of the stream (new id, block, episode, tag 3): word
// m is word m mod 4 of block m / 4.  Words 0 .. I-1 draw the immovable
// pieces among the unmoved ones (a partial shuffle from the front), words
// I .. I+L-2 shuffle the movable multiset from the back, as the oracle does.
constexpr int kUmStride = 41, kLsStride = 33;   // at least 40 unmoved pieces and 33 movable types
constexpr int kResampleRowsBytes = 64 * (kUmStride + kLsStride) * 4;

__device__ __forceinline__ void resample_wave(const ResampleSource& S, uint64_t seed, uint32_t id0, int cnt,
                                              int32_t* um, int32_t* ls, uint8_t* out) {
  const int lane = lane_id();
  int32_t* my_um = um + lane * kUmStride;
  int32_t* my_ls = ls + lane * kLsStride;
  for (int e = 0; e < S.nu; ++e) my_um[e] = __builtin_amdgcn_readlane(S.unmoved, e);
  for (int e = 0; e < S.L; ++e) my_ls[e] = __builtin_amdgcn_readlane(S.list, e);
  const uint32_t new_id = id0 + (uint32_t)lane;
  const int ndraw = S.I + (S.L > 0 ? S.L - 1 : 0);
  for (int b = 0; 4 * b < ndraw; ++b) {
    const uint4 blk = philox(make_uint4(new_id, (uint32_t)b, S.episode, 3u), seed);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = 4 * b + q;
      if (m >= ndraw) break;
      const uint32_t word = q == 0 ? blk.x : q == 1 ? blk.y : q == 2 ? blk.z : blk.w;
      int32_t* row;
      int x, y;
      if (m < S.I) {
        row = my_um;
        x = m;
        y = m + (int)mulshift(word, (uint32_t)(S.nu - m));
      } else {
        const int k = m - S.I;
        row = my_ls;
        x = S.L - 1 - k;
        y = (int)mulshift(word, (uint32_t)(S.L - k));
      }
      const int32_t vx = row[x], vy = row[y];
      row[x] = vy;
      row[y] = vx;
    }
  }
  // this lane's immovable pieces: the first nflag of the drawn ones are Flags,
  // the rest Bombs (bit m: piece 40 z + m)
  uint64_t fl = 0, bm = 0;
  for (int a = 0; a < S.I; ++a) {
    const uint64_t bit = 1ull << (my_um[a] - 40 * S.z);
    if (a < S.nflag) fl |= bit;
    else bm |= bit;
  }
  // chunk lane holds piece lane - 16 (lanes 16..63), chunk 64 + lane piece 48 + lane (lanes 0..31)
  for (int r = 0; r < cnt; ++r) {
    const uint64_t f = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(fl >> 32), r) << 32) |
                       (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)fl, r);
    const uint64_t b = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(bm >> 32), r) << 32) |
                       (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bm, r);
    const uint64_t rest = S.hidden & ~(f | b);
    const int32_t* types = ls + r * kLsStride;
    uint4 c[2] = {S.c0, S.c1};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int id = h == 0 ? lane - 16 : 48 + lane;
      const int m = id - 40 * S.z;
      const bool ours = (h == 0 ? lane >= 16 : lane < 32) && m >= 0 && m < 40;
      const int mm = ours ? m : 0;
      int t = -1;
      if (ours) {
        if ((rest >> mm) & 1ull) t = types[__popcll(rest & ((1ull << mm) - 1ull))];
        else if ((f >> mm) & 1ull) t = kFlag;
        else if ((b >> mm) & 1ull) t = kBomb;
      }
      if (t >= 0) c[h].x = (c[h].x & ~15u) | (uint32_t)t;
    }
    if (lane == 0) c[0].x = id0 + (uint32_t)r;   // header word 0: the game id
    uint4* dst = reinterpret_cast<uint4*>(out + (size_t)r * kRecordBytes);
    dst[lane] = c[0];
    if (lane < 32) dst[64 + lane] = c[1];
  }
}

// ---------------------------------------------------------------- validation
// Well-formedness of a record that did not come from this engine: lakes
// exactly on lake squares, board entries in range and alive, every alive piece
// on exactly one square, each player's types form the initial multiset, only
// movable pieces have moved, death squares/causes and ring squares in range,
// counters in range.  Everything the kernels index by record contents is
// covered, so a rejected record can never drive an out-of-range access.
__device__ __forceinline__ bool record_ok(const uint8_t* R) {
  const int lane = lane_id();
  bool bad = false;
  int my_type[2] = {-1, -1};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int s = lane + 64 * h;
    if (s < kSquares) {
      int v = board_at(R, s);
      if (is_lake_sq(s) != (v == kLake)) bad = true;
      if (v < -2 || v >= kPieces) bad = true;
      if (v >= 0 && !p_alive(piece_words(R, v)[0])) bad = true;
    }
    int id = lane + 64 * h;
    if (id < kPieces) {
      uint32_t w0 = piece_words(R, id)[0];
      int t = p_type(w0);
      my_type[h] = t;
      if (t > 11) bad = true;
      if (p_moved(w0) && !movable_type(t)) bad = true;
      if (p_long(w0) && (!p_moved(w0) || t != kScout)) bad = true;
      const int cause = (w0 >> 7) & 7, dsq = (w0 >> 10) & 127;
      if (p_alive(w0)) {
        if (cause != 0 || dsq != 127) bad = true;
        int n = 0;
        for (int s2 = 0; s2 < kSquares; ++s2) n += board_at(R, s2) == id;
        if (n != 1) bad = true;
      } else {
        if (cause < 1 || cause > 6 || dsq >= kSquares || !p_revealed(w0)) bad = true;
      }
    }
    if (lane < 64) {
      int b = R[kOffRing + lane];
      if (b >= kSquares) bad = true;
    }
  }
  // per-player type multiset equals the initial one (Table "pieces")
  for (int t = 0; t < 12; ++t) {
    uint64_t a = ballot(my_type[0] == t);   // ids 0..63
    uint64_t b = ballot(my_type[1] == t);   // ids 64..79 in lanes 0..15
    int red = __popcll(a & 0xFFFFFFFFFFull);
    int blue = __popcll(a >> 40) + __popcll(b & 0xFFFFull);
    if (red != initial_count(t) || blue != initial_count(t)) bad = true;
  }
  if (R[kOffRingCount] > 32 || R[kOffDone] > 1 || R[kOffReason] > 5 ||
      (int)hdr_u32(R, kOffPly) < 0 || (int)hdr_u32(R, kOffPly) > 32767 ||
      (int)hdr_u32(R, kOffBattleless) < 0)
    bad = true;
  // chase: a chasing player only while a chase lasts
  if (R[kOffChaser] > 1 || (R[kOffChaseLen] == 0 && R[kOffChaser] != 0)) bad = true;
  // two-square records: 0 or 2-4 squares on the board, of a piece id of that
  // player, unused bytes zero
  if (lane < 2) {
    const uint8_t* t = R + kOffTwoSquare + 8 * lane;
    if (t[1] > 4 || t[1] == 1) bad = true;
    if (t[1] > 0 ? (t[0] >= kPieces || owner(t[0]) != lane) : t[0] != 0) bad = true;
    for (int i = 0; i < 4; ++i)
      if (i < t[1] ? t[2 + i] >= kSquares : t[2 + i] != 0) bad = true;
  }
  return ballot(bad) == 0;
}

}  // namespace sg
