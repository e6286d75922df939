// libstratego.so: kernels and the C ABI declared in include/stratego.h.
//
// Plain engine: one launch per call (legal mask, sample, step, encode), one
// wavefront per game, four games per 256-thread workgroup.
// Fused engine: one persistent kernel per ply (mask -> sample -> encode ->
// step), grid sized to the device's occupancy, each wave working through
// tiles of G consecutive games, plies optionally replayed from a captured
// hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "stratego.h"
#include "device.h"

using namespace sg;

namespace {

enum : int { kDoMask = 1, kDoSample = 2, kDoEncode = 4, kDoStep = 8, kStepFromInput = 16 };
constexpr int kFused = kDoMask | kDoSample | kDoEncode | kDoStep;
constexpr int kMaxTimedPlies = 4096;
constexpr int kMaxHistory = 1 << 20;

struct PlyArgs {
  uint8_t* states;
  const int32_t* slots;
  int32_t n;
  int32_t total;      // games in the context (slot range)
  int32_t out_base;   // index of this ply's row in [nplies][n] outputs
  const int32_t* out_index;   // output row of game i (NULL: i)
  uint64_t* mask;
  int16_t* num_legal;
  const int16_t* actions_in;
  int16_t* actions_out;
  uint8_t* obs;
  int8_t* done;
  int8_t* outcome;
  uint8_t* reason;
  int16_t* ep_len;
  int32_t* err;
  unsigned long long* ts;
  unsigned int* tickets;   // this ply's work counter (plies with observations), else NULL
  // rollout buffer: record and step outcome of every stepped game at
  // row *hist_slot of the ring (NULL: not recorded)
  uint8_t* hist;
  uint64_t* hist_steps;
  const int32_t* hist_slot;
  Rules rules;
  int32_t games_per_tile;
  int32_t tail_from;  // tiles from this one on hold one game each (-1: none)
  int32_t layout;     // observation staging layout in LDS
};

// Step outcome of one game at one time step of the rollout buffer: action
// (bits 0-15), done (16-23), outcome (24-31), reason (32-39), ep_len (48-63).
__device__ __forceinline__ uint64_t pack_step(int action, const StepOut& o) {
  return (uint64_t)(uint16_t)(int16_t)action | (uint64_t)(uint8_t)o.done << 16 |
         (uint64_t)(uint8_t)(int8_t)o.outcome << 24 | (uint64_t)(uint8_t)o.reason << 32 |
         (uint64_t)(uint16_t)(int16_t)o.ep_len << 48;
}

// Per-wave LDS: the slab of the layout plus a spare record buffer.  While a
// game is processed, the next game's record is fetched into registers early
// and parked in the spare buffer before the observation stream starts, so no
// global load is waited on right after a burst of stores (on gfx950 one
// counter tracks both, and waiting for a load would also drain the stores).
__host__ __device__ __forceinline__ constexpr int wave_lds_bytes(int layout) { return slab_bytes_for(layout) + kRecordBytes; }

// ENC: 0 byte images (layouts 2-6), 1 bit planes of both observers (layout 1),
// 2 bit planes of one observer at a time (layout 7), 3 no observations: plies
// that only mask, sample and step (rollouts, recording plies).  Those need
// only the record, the work areas and the to-square sets (4.9 KB of LDS per
// wave with the spare record), so a CU holds 32 of their waves instead of the
// 8 the both-observer encoder allows.  Register budgets: the both-observer
// encoder is LDS-bound at 2 waves per SIMD anyway, so it may use 256 VGPRs;
// the one-observer encoder runs best at 3 (168 VGPRs, no spills; 4% faster
// than 4 waves with 128 and spills); the observation-free register-board
// variant without a mask output at 7 (72 VGPRs, no spills; 3% faster than 8
// waves with 64 VGPRs and a few spilled), the other observation-free ones at
// 5 (96 VGPRs, the general one with a few spilled); the byte-image layouts
// at 4.
constexpr int kEncNone = 3;
constexpr int kNoObsSlabBytes = kSlabImage + kDestSetBytes;
__host__ __device__ __forceinline__ constexpr int ply_slab_bytes(int enc, int layout) {
  return enc == kEncNone ? kNoObsSlabBytes : slab_bytes_for(layout);
}
__host__ __device__ __forceinline__ constexpr int ply_wave_lds_bytes(int enc, int layout) {
  return ply_slab_bytes(enc, layout) + kRecordBytes;
}
static_assert(kNoObsSlabBytes % 16 == 0, "record buffers stay 16-byte aligned");

// An entry of an index list at a wave-uniform position, read through the
// scalar unit (the lists are not written during a launch), so that no wait on
// the vector-memory counter, which also holds the stores in flight, is needed
// for it.
__device__ __forceinline__ int32_t uniform_load(const int32_t* list, int idx) {
  idx = __builtin_amdgcn_readfirstlane(idx);
  return ((const __attribute__((address_space(4))) int32_t*)list)[idx];
}

// The ply kernel's argument block (its only argument, at offset 0 of the
// argument segment) through an address the compiler cannot carry from one
// loop iteration to the next.  Pointers a game uses once, for its output rows,
// are read through it where they are used: one scalar load.  Read through the
// by-value argument instead, they are hoisted out of the per-game loop, and
// with scalar registers short the register allocator spills them to vector
// lanes and reads them back, one vector instruction per 32 bits, on every
// game.  Only for use inside k_ply.
__device__ __forceinline__ const __attribute__((address_space(4))) PlyArgs* args_fresh() {
  uint64_t p = (uint64_t)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return (const __attribute__((address_space(4))) PlyArgs*)p;
}

// The rules, read field by field through args_fresh (a struct copy out of
// the constant address space has no constructor).  Observation-free plies
// read them per game: held for the whole launch, they pushed other scalar
// values into spills.
__device__ __forceinline__ Rules rules_fresh() {
  const auto* f = args_fresh();
  Rules r;
  r.seed = f->rules.seed;
  r.k_battleless = f->rules.k_battleless;
  r.max_moves = f->rules.max_moves;
  r.auto_reset = f->rules.auto_reset;
  r.two_square = f->rules.two_square;
  r.sampler = f->rules.sampler;
  r.chasing = f->rules.chasing;
  r.acting_obs = f->rules.acting_obs;
  return r;
}

// A record as two 768-byte halves, 12 bytes per lane: every lane takes part
// in both accesses, so no branch can skip one.  (A skipped access would leave
// the compiler unsure which loads are still in flight, and it would then wait
// for all of them, stores included.)
struct __attribute__((aligned(4))) Rec12 {
  uint32_t x, y, z;
};
struct RecRegs {
  Rec12 lo, hi;
};
__device__ __forceinline__ RecRegs rec_load(const uint8_t* g) {
  const int lane = lane_id();
  const Rec12* src = reinterpret_cast<const Rec12*>(g);
  return RecRegs{src[lane], src[64 + lane]};
}
__device__ __forceinline__ void rec_store(uint8_t* g, const RecRegs& r) {
  const int lane = lane_id();
  Rec12* dst = reinterpret_cast<Rec12*>(g);
  dst[lane] = r.lo;
  dst[64 + lane] = r.hi;
}

// A game's mask words and legal-move count.
__device__ __forceinline__ void store_mask_outputs(int oi, const uint64_t w[3], int n, bool with_mask) {
  const int lane = lane_id();
  uint64_t* const mask = args_fresh()->mask;
  if (with_mask && mask) {
    uint64_t* m = mask + (size_t)oi * kMaskWords;
#pragma unroll
    for (int g = 0; g < 3; ++g)
      if (lane + 64 * g < kMaskWords) m[lane + 64 * g] = w[g];
  }
  if (lane == 0) {
    int16_t* const num_legal = args_fresh()->num_legal;
    if (num_legal) num_legal[oi] = (int16_t)n;
  }
}

// FAST: the fused ply's register-board path (drawn actions, neither
// competitive-play rule on); otherwise the general path.  NOMASK: no mask
// output (a.mask is NULL), so the ply samples from move counts alone.
template <int MODE, int ENC, bool FAST = false, bool NOMASK = false>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(ENC == 1 ? 2 : ENC == 2 ? 3 : ENC == kEncNone ? (FAST && NOMASK ? 7 : 5) : 4))) k_ply(PlyArgs a) {
  static_assert(!FAST || MODE == (kDoMask | kDoSample | kDoEncode | kDoStep), "the fast path is the fused ply's");
  static_assert(FAST || !NOMASK, "the mask-free variant is a fast-path one");
  extern __shared__ __align__(16) uint8_t smem[];
  const int W = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = lane_id();
  uint8_t* slab = smem + wave * ply_wave_lds_bytes(ENC, a.layout);
  // the two record buffers are slab + 0 and slab + spare; offsets (not a
  // pointer array) keep every access an LDS instruction
  const int spare = ply_slab_bytes(ENC, a.layout);
  if (a.ts && threadIdx.x == 0) atomicMin(&a.ts[0], (unsigned long long)wall_clock64());
  const bool encode = ENC != kEncNone && (MODE & kDoEncode) && a.obs;
  const size_t hist_row = ((MODE & kDoStep) && a.hist) ? (size_t)(*a.hist_slot) * (size_t)a.total : 0;
  const bool byte_image = encode && ENC == 0;
  if (byte_image) clear_lds(slab + kSlabImage, image_bytes_for(a.layout));
  const int G = a.games_per_tile;
  // tiles below T1 hold G games, the ones from T1 on a single game (with
  // tickets, the last tiles handed out are single games, so the ply does not
  // end on a few waves finishing long tiles)
  // (only plies with observations take tiles from tickets)
  constexpr bool kTail = ENC != kEncNone;
  const int T1 = (kTail && a.tail_from >= 0) ? a.tail_from : INT_MAX;
  const int ntiles = (kTail && a.tail_from >= 0) ? T1 + (a.n - T1 * G) : (a.n + G - 1) / G;
  auto tfirst = [&](int t) {
    if constexpr (kTail) return t < T1 ? t * G : T1 * G + (t - T1);
    else return t * G;
  };
  auto tlen = [&](int t) {
    if constexpr (kTail) return t < T1 ? G : 1;
    else return G;
  };
  // Work distribution: every wave works through tiles of G consecutive games
  // of its own.  With a ticket counter (persistent plies with observations) a
  // wave takes the next tile in address order whenever it becomes free;
  // otherwise wave w of workgroup b takes tiles bW+w, bW+w+gridDim.x*W, ...
  const bool dynamic = ENC != kEncNone && a.tickets != nullptr;   // plies without observations split statically
  const int workers = gridDim.x * W;
  auto grab = [&]() -> int {
    int t = 0;
    if (lane == 0) t = (int)atomicAdd(a.tickets, 1u);
    return __shfl(t, 0, 64);
  };
  int tile = dynamic ? grab() : (int)blockIdx.x * W + wave;
  // Observation-free plies draw their actions ahead.  Games are split
  // statically, so a wave knows which games it will take, and a launch steps
  // each game once, from the counter (game id, ply, episode) its record holds
  // when the launch starts.  Lane j computes the generator's block for the
  // wave's j-th game: one pass on the vector unit covers 64 games, where a
  // pass per game on the scalar unit was ten rounds of multiplies each.  A
  // wave's games beyond the 64th draw in the loop as before.  (The counters
  // are read while no store is in flight, at the top of the launch.)
  constexpr bool kAhead = ENC == kEncNone && FAST;
  uint4 ahead = make_uint4(0u, 0u, 0u, 0u);   // words x, y, z of this lane's game
  int kcur = 0;                               // this wave's games so far
  if constexpr (kAhead) {
    const int t = tile + (lane / G) * workers;
    const int ii = t < ntiles ? t * G + lane % G : a.n;
    uint4 c = make_uint4(0u, 0u, 0u, 0u);
    if (ii < a.n) {
      const int sl = a.slots ? a.slots[ii] : ii;
      if (sl >= 0 && sl < a.total) {
        const uint4 h = *reinterpret_cast<const uint4*>(a.states + (size_t)sl * kRecordBytes);
        static_assert(kOffGameId == 0 && kOffEpisode == 4 && kOffPly == 8, "the counter is the header's first words");
        c = make_uint4(h.x, h.z, h.y, 0u);   // game id, ply, episode
      }
    }
    ahead = philox(c, a.rules.seed);
  }
  int gi = 0;
  int i = tile < ntiles ? tfirst(tile) + gi : a.n;
  bool have = i < a.n;
  int slot = have ? (a.slots ? uniform_load(a.slots, i) : i) : 0;
  bool slot_ok = have && slot >= 0 && slot < a.total;
  if (slot_ok) load_record(slab, a.states + (size_t)slot * kRecordBytes);
  int cur = 0;   // offset of the current record buffer: 0 or spare
  // Plies without observations write a game's record back only once the
  // next game's record has arrived: one counter tracks loads and stores in
  // issue order, so a wait for a load also waits for every store issued
  // before it.  The pending record sits in the other buffer until the next
  // record is parked there; it is read into registers first and stored after
  // the park, so that no wait follows these stores within the game.  (The
  // few bytes of per-game results are stored right after the step.)
  constexpr bool kDefer = ENC == kEncNone && (MODE & kDoStep) != 0;
  uint8_t* pend_g = nullptr;    // where the pending record goes (NULL: none)
  auto flush = [&](const RecRegs& r) {
    if (!kDefer || pend_g == nullptr) return;
    rec_store(pend_g, r);
    pend_g = nullptr;
  };
  while (have) {
    // the next game of this wave (its chunk is grabbed only when needed)
    int ngi = gi + 1, ntile = tile;
    bool need_grab = false;
    if (ngi >= tlen(tile) || tfirst(tile) + ngi >= a.n) {
      ngi = 0;
      if (dynamic) need_grab = true;
      else ntile += workers;
    }
    int inext = a.n;
    bool next_have = false, resolved = false;
    int next_slot = 0;
    bool next_ok = false;
    auto resolve_next = [&]() {
      if (resolved) return;
      resolved = true;
      if (need_grab) ntile = grab();
      inext = ntile < ntiles ? tfirst(ntile) + ngi : a.n;
      next_have = inext < a.n;
      if (next_have) {
        next_slot = a.slots ? uniform_load(a.slots, inext) : inext;
        next_ok = next_slot >= 0 && next_slot < a.total;
      }
    };
    if (!need_grab) resolve_next();
    uint4 p0 = make_uint4(0, 0, 0, 0), p1 = make_uint4(0, 0, 0, 0);
    RecRegs pn{};
    bool fetched = false;
    auto fetch_next = [&]() {
      resolve_next();
      if (next_ok && !fetched) {
        const uint8_t* g = a.states + (size_t)next_slot * kRecordBytes;
        if (kDefer) {
          pn = rec_load(g);
        } else {
          const uint4* src = reinterpret_cast<const uint4*>(g);
          p0 = src[lane];
          if (lane < 32) p1 = src[64 + lane];
        }
      }
      fetched = true;
    };
    bool parked = false;
    auto park_next = [&]() {
      fetch_next();
      if constexpr (kDefer) {
        if (parked) return;
        parked = true;
        uint8_t* spare_buf = slab + (spare - cur);
        // the previous game's record leaves the spare buffer before the next
        // one is parked there (zeros when there is no next game), and is
        // stored only after that park
        RecRegs r{};
        if (pend_g != nullptr) r = rec_load(spare_buf);
        rec_store(spare_buf, pn);
        flush(r);
      } else {
        if (next_ok && !parked) {
          uint4* dst = reinterpret_cast<uint4*>(slab + (spare - cur));
          dst[lane] = p0;
          if (lane < 32) dst[64 + lane] = p1;
        }
        parked = true;
      }
    };
    if (!slot_ok) {
      if (lane == 0) atomicMin(&a.err[1], i);
      park_next();
    } else {
      uint8_t* R = slab + cur;
      uint8_t* gstate = a.states + (size_t)slot * kRecordBytes;
      const int32_t* const out_index = args_fresh()->out_index;
      const int oi = out_index ? uniform_load(out_index, i) : i;
      int action = -1;
      SquareRegs rg;
      uint64_t w[3];
      int n;
      if (MODE & kDoMask) {
        uint64_t d[4];
        uint32_t pk[2];
        if (FAST) {
          // with a mask to write, the destination sets; else counts suffice
          load_regs(R, rg);
          const int p = (int)(uniform_u32(hdr_u32(R, kOffPly)) & 1);
          const bool done = uniform_u32(R[kOffDone]) != 0;
          if (!NOMASK && a.mask) {
            fast_dests(rg, p, done, d);
            n = count_dests(d);
            words_from_dests(d, reinterpret_cast<uint64_t*>(slab + kSlabImage), w);
          } else {
            dir_counts(rg, p, done, pk);
            n = total_count(pk);
          }
        } else {
          n = legal_mask_words(R, reinterpret_cast<uint64_t*>(slab + kSlabImage), w, a.rules, slab + kSlabProbQ);
        }
        fetch_next();
        if (!kDefer) {
          if (!NOMASK && a.mask) {
            uint64_t* m = a.mask + (size_t)oi * kMaskWords;
#pragma unroll
            for (int g = 0; g < 3; ++g)
              if (lane + 64 * g < kMaskWords) m[lane + 64 * g] = w[g];
          }
          if (a.num_legal && lane == 0) a.num_legal[oi] = (int16_t)n;
        }
        if (FAST && (MODE & kDoSample)) {
          // wave-uniform copies of the counter, so that the generator (unless
          // the draw was taken ahead) and the selection run on the scalar unit
          uint32_t gid = 0, ply = 0, ep = 0;
          if constexpr (!kAhead) {
            gid = uniform_u32(hdr_u32(R, kOffGameId));
            ply = uniform_u32(hdr_u32(R, kOffPly));
            ep = uniform_u32(hdr_u32(R, kOffEpisode));
          }
          auto draw = [&]() -> uint4 {
            if constexpr (kAhead) {
              if (kcur < 64)
                return make_uint4((uint32_t)__builtin_amdgcn_readlane((int)ahead.x, kcur),
                                  (uint32_t)__builtin_amdgcn_readlane((int)ahead.y, kcur),
                                  (uint32_t)__builtin_amdgcn_readlane((int)ahead.z, kcur), 0u);
              return philox(make_uint4(uniform_u32(hdr_u32(R, kOffGameId)), uniform_u32(hdr_u32(R, kOffPly)),
                                       uniform_u32(hdr_u32(R, kOffEpisode)), 0u),
                            args_fresh()->rules.seed);
            } else {
              return philox(make_uint4(gid, ply, ep, 0u), a.rules.seed);
            }
          };
          const bool magnet = (kAhead ? args_fresh()->rules.sampler : a.rules.sampler) == kSamplerMagnet;
          if (!NOMASK && a.mask)
            action = magnet ? (n == 0 ? -1 : sample_magnet(d[0], d[1], d[2], d[3], draw)) : sample_dests(d, n, draw);
          else
            action = magnet ? (n == 0 ? -1 : magnet_counts(pk, draw)) : sample_counts(pk, n, draw);
          if (!kDefer && a.actions_out && lane == 0) a.actions_out[(size_t)a.out_base + oi] = (int16_t)action;
        } else if (MODE & kDoSample) {
          if (a.rules.sampler == kSamplerMagnet) {
            const uint64_t* ts = reinterpret_cast<const uint64_t*>(slab + kSlabImage);
            const bool second = lane + 64 < kSquares;
            action = n == 0 ? -1
                            : sample_magnet(ts[2 * lane], ts[2 * lane + 1], second ? ts[2 * lane + 128] : 0ull,
                                            second ? ts[2 * lane + 129] : 0ull, a.rules.seed,
                                            hdr_u32(R, kOffGameId), hdr_u32(R, kOffPly), hdr_u32(R, kOffEpisode));
          } else {
            action = sample_from_words(w, n, a.rules.seed, hdr_u32(R, kOffGameId),
                                       hdr_u32(R, kOffPly), hdr_u32(R, kOffEpisode));
          }
          if (!kDefer && a.actions_out && lane == 0) a.actions_out[(size_t)a.out_base + oi] = (int16_t)action;
        }
        wave_sync();
        if (byte_image) clear_lds(slab + kSlabImage, kDestSetBytes);
      }
      park_next();
      if (kDefer && (MODE & kDoMask)) {   // this game's mask outputs, behind the park
        store_mask_outputs(oi, w, n, !NOMASK);
        if ((MODE & kDoSample) && lane == 0) {
          int16_t* const actions_out = args_fresh()->actions_out;
          if (actions_out) actions_out[(size_t)a.out_base + oi] = (int16_t)action;
        }
      }
      if (MODE & kStepFromInput) action = a.actions_in[i];
      if (encode) {
        compute_probq(R, slab);
        uint8_t* out = a.obs + (size_t)oi * obs_bytes_per_game(a.rules);
        if (ENC == 1) encode_game_bits(R, slab, a.rules, out);
        else if (ENC == 2) encode_game_bits1(R, slab, a.rules, out);
        else encode_game_bytes(R, slab, a.rules, segments_of(a.layout), out);
      }
      if (MODE & kDoStep) {
        uint8_t* const hist = args_fresh()->hist;
        if (hist) store_record(hist + (hist_row + slot) * kRecordBytes, R);   // the state acted on
        StepOut o = FAST ? fast_step_game(R, slab + kSlabScratch, slab + kSlabProbQ, kAhead ? rules_fresh() : a.rules, action, rg)
                         : step_game<(MODE & kStepFromInput) != 0>(R, slab + kSlabScratch, slab + kSlabProbQ,
                                                                    a.rules, action);
        const size_t row = (size_t)a.out_base + oi;
        if (lane == 0) {
          const auto* f = args_fresh();
          int8_t* const done_p = f->done;
          int8_t* const outcome_p = f->outcome;
          uint8_t* const reason_p = f->reason;
          int16_t* const ep_len_p = f->ep_len;
          if (done_p) done_p[row] = (int8_t)o.done;
          if (outcome_p) outcome_p[row] = (int8_t)o.outcome;
          if (reason_p) reason_p[row] = (uint8_t)o.reason;
          if (ep_len_p) ep_len_p[row] = (int16_t)o.ep_len;
          if (o.illegal) atomicMin(&f->err[0], slot);
          if (f->hist) f->hist_steps[hist_row + slot] = pack_step(action, o);
        }
        wave_sync();
        if (kDefer) {
          pend_g = gstate;
        } else {
          store_record(gstate, R);
        }
      }
    }
    resolve_next();
    wave_sync();
    i = inext;
    tile = ntile;
    gi = ngi;
    ++kcur;
    slot = next_slot;
    slot_ok = next_ok;
    have = next_have;
    cur = spare - cur;
  }
  if (kDefer && pend_g != nullptr) flush(rec_load(slab + (spare - cur)));   // the last game's write-back
  if (a.ts) {
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&a.ts[1], (unsigned long long)wall_clock64());
  }
}

// Uniform legal action from a caller-supplied mask (plain engine).
__global__ void __launch_bounds__(256) k_sample(const uint8_t* states, int32_t n, const uint64_t* mask,
                                               const int16_t* num_legal, int16_t* actions, uint64_t seed,
                                               int32_t sampler) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int i = blockIdx.x * (blockDim.x >> 6) + wave;
  if (i >= n) return;
  const uint8_t* g = states + (size_t)i * kRecordBytes;
  const uint32_t game_id = *reinterpret_cast<const uint32_t*>(g + kOffGameId);
  const uint32_t episode = *reinterpret_cast<const uint32_t*>(g + kOffEpisode);
  const uint32_t ply = *reinterpret_cast<const uint32_t*>(g + kOffPly);
  const bool done = g[kOffDone] != 0;
  uint64_t w[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int word = lane + 64 * k;
    w[k] = word < kMaskWords ? mask[(size_t)i * kMaskWords + word] : 0ull;
  }
  const int nl = done ? 0 : num_legal[i];
  int action;
  if (sampler == kSamplerMagnet) {
    const uint64_t* m = mask + (size_t)i * kMaskWords;
    uint64_t lo0, hi0, lo1, hi1;
    square_set_from_mask(m, lane, lo0, hi0);
    square_set_from_mask(m, lane + 64, lo1, hi1);
    action = nl == 0 ? -1 : sample_magnet(lo0, hi0, lo1, hi1, seed, game_id, ply, episode);
  } else {
    action = sample_from_words(w, nl, seed, game_id, ply, episode);
  }
  if (lane == 0) actions[i] = (int16_t)action;
}

// Fresh setups (episode 0) for the listed slots.
__global__ void __launch_bounds__(256) k_reset_fresh(uint8_t* states, const int32_t* slots, int32_t n,
                                                    int32_t total, Rules rules, uint32_t game_id_base,
                                                    int32_t* err) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = threadIdx.x >> 6;
  const int i = blockIdx.x * (blockDim.x >> 6) + wave;
  if (i >= n) return;
  uint8_t* slab = smem + wave * kSlabImage;
  const int slot = slots ? slots[i] : i;
  if (slot < 0 || slot >= total) {
    if (lane_id() == 0) atomicMin(&err[1], i);
    return;
  }
  reset_game(slab, slab + kSlabScratch, slab + kSlabProbQ, rules, game_id_base + (uint32_t)slot, 0u, 0u);
  store_record(states + (size_t)slot * kRecordBytes, slab);
}

// Import caller records into the listed slots after a well-formedness check.
__global__ void __launch_bounds__(256) k_import(uint8_t* states, const int32_t* slots, int32_t n,
                                               int32_t total, const uint8_t* src, int32_t* err) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = threadIdx.x >> 6;
  const int i = blockIdx.x * (blockDim.x >> 6) + wave;
  if (i >= n) return;
  uint8_t* R = smem + wave * kSlabImage;
  const int slot = slots ? slots[i] : i;
  if (slot < 0 || slot >= total) {
    if (lane_id() == 0) atomicMin(&err[1], i);
    return;
  }
  load_record(R, src + (size_t)i * kRecordBytes);
  if (record_ok(R)) store_record(states + (size_t)slot * kRecordBytes, R);
  else if (lane_id() == 0) atomicMin(&err[1], slot);
}

// Slot k = i*per + j receives a resample of source record i.  Each wave takes
// up to 64 consecutive resamples of one source, one per lane: it loads and
// checks the source once, draws the resamples in its lanes, then stores them.
constexpr int kResamplesPerWave = 64;
constexpr int kResampleWaves = 4;   // waves per workgroup
constexpr int kResampleWaveBytes = kRecordBytes + kResampleRowsBytes;
__global__ void __launch_bounds__(64 * kResampleWaves) k_resample(uint8_t* states, const uint8_t* src,
                                                                 int32_t nsrc, int32_t per, uint64_t seed,
                                                                 uint32_t id_base, int32_t* err) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = threadIdx.x >> 6;
  const int chunks = (per + kResamplesPerWave - 1) / kResamplesPerWave;
  const int64_t w = (int64_t)blockIdx.x * kResampleWaves + wave;
  if (w >= (int64_t)nsrc * chunks) return;
  const int i = (int)(w / chunks);
  const int j0 = (int)(w % chunks) * kResamplesPerWave;
  const int cnt = per - j0 < kResamplesPerWave ? per - j0 : kResamplesPerWave;
  uint8_t* R = smem + wave * kResampleWaveBytes;
  int32_t* um = reinterpret_cast<int32_t*>(R + kRecordBytes);
  load_record(R, src + (size_t)i * kRecordBytes);
  if (!record_ok(R)) {
    if (lane_id() == 0) atomicMin(&err[1], i * per + j0);
    return;
  }
  const ResampleSource S = resample_prepare(R);
  const int k0 = i * per + j0;
  resample_wave(S, seed, id_base + (uint32_t)k0, cnt, um, um + 64 * kUmStride, states + (size_t)k0 * kRecordBytes);
}

// Copy the records of the listed slots to out (contiguous).
__global__ void __launch_bounds__(256) k_gather(const uint8_t* states, const int32_t* slots, int32_t n,
                                               uint8_t* out) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int i = blockIdx.x * (blockDim.x >> 6) + wave;
  if (i >= n) return;
  const uint4* src = reinterpret_cast<const uint4*>(states + (size_t)slots[i] * kRecordBytes);
  uint4* dst = reinterpret_cast<uint4*>(out + (size_t)i * kRecordBytes);
  dst[lane] = src[lane];
  if (lane < 32) dst[64 + lane] = src[64 + lane];
}

__global__ void k_ts_init(unsigned long long* ts, int32_t nplies) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nplies) {
    ts[2 * i] = ~0ull;
    ts[2 * i + 1] = 0ull;
  }
}

__global__ void k_ts_convert(const unsigned long long* ts, int32_t nplies, double ns_per_tick,
                             int64_t* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nplies) out[i] = (int64_t)((double)(ts[2 * i + 1] - ts[2 * i]) * ns_per_tick);
}

// Copy of n words, here from pinned host memory through its device mapping:
// on the compute stream itself, so no copy engine has to hand over to it.
__global__ void k_copy_i32(int32_t* dst, const int32_t* src, int32_t n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_fill_i32(int32_t* p, int32_t n, int32_t v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Rows of the rollout buffer's ring for the next nplies recorded plies, from
// the device's time-step counter, which then advances.  A kernel, so that
// every replay of a captured graph takes fresh rows.
__global__ void __launch_bounds__(256) k_hist_clock(int64_t* clock, int32_t* rows, int32_t nplies,
                                                   int32_t H) {
  const int64_t t = clock[0];
  for (int p = threadIdx.x; p < nplies; p += blockDim.x) rows[p] = (int32_t)((t + p) % H);
  __syncthreads();
  if (threadIdx.x == 0) clock[0] = t + nplies;
}

// ---------------------------------------------------------------- rollout-buffer queries
// App. B.1: quantities of a past time step are recomputed from the recorded
// state instead of being stored.  One wave per listed game.
enum : int { kQMask = 0, kQObs = 1, kQInfo = 2, kQRecord = 3 };

struct HistArgs {
  const uint8_t* src;       // records at time step t: a ring row or the live states
  const uint64_t* steps;    // step outcomes at t (NULL: t is the current step)
  const uint8_t* ring;      // the whole ring, for walking back over earlier steps
  int64_t t, oldest;
  int32_t H, N;
  const int32_t* games;     // games to query (NULL: 0..count-1)
  int32_t count;
  uint64_t* mask;
  int16_t* num_legal;
  uint8_t* obs;
  uint8_t* records;
  stratego_history_outputs out;
  int32_t* err;
  Rules rules;
};

__host__ __device__ __forceinline__ constexpr int hist_lds_bytes(int q) {
  return q == kQObs ? slab_bytes_for(kLayoutBits)
       : q == kQMask ? kSlabImage + kDestSetBytes
       : q == kQInfo ? kSlabImage : 16;
}

template <int Q>
__global__ void __launch_bounds__(256) k_hist(HistArgs h) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int i = blockIdx.x * (blockDim.x >> 6) + wave;
  if (i >= h.count) return;
  const int g = h.games ? h.games[i] : i;
  if (g < 0 || g >= h.N) {
    if (lane == 0) atomicMin(&h.err[1], i);
    return;
  }
  const uint8_t* src = h.src + (size_t)g * kRecordBytes;
  if (Q == kQRecord) {
    store_record(h.records + (size_t)i * kRecordBytes, src);
    return;
  }
  uint8_t* slab = smem + wave * hist_lds_bytes(Q);
  uint8_t* R = slab;
  load_record(R, src);
  if (Q == kQMask) {
    uint64_t w[3];
    const int n = legal_mask_words(R, reinterpret_cast<uint64_t*>(slab + kSlabImage), w, h.rules, slab + kSlabProbQ);
    if (h.mask) {
      uint64_t* m = h.mask + (size_t)i * kMaskWords;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (lane + 64 * k < kMaskWords) m[lane + 64 * k] = w[k];
    }
    if (h.num_legal && lane == 0) h.num_legal[i] = (int16_t)n;
  } else if (Q == kQObs) {
    compute_probq(R, slab);
    encode_game_bits(R, slab, h.rules, h.obs + (size_t)i * obs_bytes_per_game(h.rules));
  } else {
    const stratego_history_outputs& o = h.out;
    const int ply = (int)hdr_u32(R, kOffPly), p = ply & 1;
    const bool done = R[kOffDone] != 0;
    const bool movable = has_move(R, p, h.rules, slab + kSlabProbQ) && !done;   // wave-wide
    // per-square views in the acting player's frame
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int sq = lane + 64 * k;
      if (sq >= kSquares) break;
      const int f = p == 0 ? sq : 99 - sq;
      const int id = board_at(R, sq);
      int plane = -1;
      bool unknown = false;
      if (id >= 0) {
        const uint32_t w0 = piece_words(R, id)[0];
        const bool own = owner(id) == p;
        plane = (own ? 0 : 12) + p_type(w0);
        unknown = !own && !p_revealed(w0);
      }
      if (o.is_unknown) o.is_unknown[(size_t)i * kSquares + f] = (uint8_t)unknown;
      if (o.piece_onehot)
        for (int c = 0; c < 24; ++c) o.piece_onehot[((size_t)i * 24 + c) * kSquares + f] = (uint8_t)(c == plane);
    }
    if (lane == 0) {
      int action = -1, sdone = 0, soutcome = 0, sreason = 0;
      if (h.steps) {
        const uint64_t e = h.steps[g];
        action = (int16_t)(e & 0xffffu);
        sdone = (int)((e >> 16) & 0xffu);
        soutcome = (int8_t)((e >> 24) & 0xffu);
        sreason = (int)((e >> 32) & 0xffu);
      }
      const bool ended = sdone && !done;   // the action at t ended the episode
      int since = 0;
      if (done) {   // steps since the episode ended: the run of terminal states up to t
        since = 1;
        for (int64_t u = h.t - 1; u >= h.oldest; --u) {
          const uint8_t* e = h.ring + ((size_t)(u % h.H) * h.N + g) * kRecordBytes;
          if (!e[kOffDone]) break;
          ++since;
        }
      }
      if (o.acting_player) o.acting_player[i] = (int8_t)p;
      if (o.played_action) o.played_action[i] = (int16_t)action;
      if (o.num_moves) o.num_moves[i] = ply;
      if (o.moves_since_attack) o.moves_since_attack[i] = (int32_t)hdr_u32(R, kOffBattleless);
      if (o.reward_pl0) o.reward_pl0[i] = (int8_t)(ended ? soutcome : 0);
      if (o.terminated_since) o.terminated_since[i] = since;
      if (o.has_legal_movement) o.has_legal_movement[i] = (uint8_t)movable;
      if (o.flag_captured) o.flag_captured[i] = (uint8_t)(ended && sreason == kReasonFlag);
      if (o.two_square_applies) {   // the rule removes a move the acting player could otherwise make
        bool applies = false;
        int x, axis, L, H;
        if (h.rules.two_square && !done && two_square_window(R, p, x, axis, L, H)) {
          uint64_t lo, hi;
          destinations(R, x, p, lo, hi);
          const uint64_t lo0 = lo, hi0 = hi;
          two_square_clear(x, axis, L, H, lo, hi);
          applies = lo != lo0 || hi != hi0;
        }
        o.two_square_applies[i] = (uint8_t)applies;
      }
      if (o.chase_applies) {   // the chasing rule removes a move the acting player could otherwise make
        bool applies = false;
        if (h.rules.chasing && !done && chase_active(R, p)) {
          uint8_t* work = slab + kSlabProbQ;
          const int nf = chase_forbidden_list(R, p, work);
          for (int k = 0; k < nf && !applies; ++k) {
            uint64_t lo, hi;
            const int x = work[kWorkFrom + k], y = work[kWorkTo + k];
            destinations(R, x, p, lo, hi);
            int x2, axis, L, H;
            if (h.rules.two_square && two_square_window(R, p, x2, axis, L, H) && x2 == x)
              two_square_clear(x, axis, L, H, lo, hi);
            applies = ((y < 64 ? lo >> y : hi >> (y - 64)) & 1) != 0;
          }
        }
        o.chase_applies[i] = (uint8_t)applies;
      }
    }
  }
}

// ---------------------------------------------------------------- policies over legal lists
// Section 2.4 / App. D.4 (magnet policy) and section 2.5 / App. D.7 (search policy).  A
// game's legal list is its legal actions in ascending order, padded to
// kMaxLegal with -1; per-action inputs and outputs are aligned with it.
enum : int { kPList = 0, kPMagnet = 1, kPSearch = 2, kPSample = 3 };

struct PolicyArgs {
  const uint8_t* states;
  int32_t n;
  int16_t* actions;        // list (kPList) or sampled action (kPSample)
  int16_t* num_legal;
  float* probs;            // kPMagnet / kPSearch output
  const float* q;          // kPSearch: advantage estimates per listed action
  const float* logpi;      // kPSearch: log of the network policy per listed action
  const float* in_probs;   // kPSample: distribution per listed action
  float alpha, beta;
  Rules rules;
};

constexpr int kPolicyList = kSlabImage + kDestSetBytes;   // int16 [kMaxLegal] in LDS
__host__ __device__ __forceinline__ constexpr int policy_lds_bytes() { return kPolicyList + 2 * kMaxLegal; }

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  return v;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <int Q>
__global__ void __launch_bounds__(256) k_policy(PolicyArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int i = blockIdx.x * (blockDim.x >> 6) + wave;
  if (i >= a.n) return;
  uint8_t* slab = smem + wave * policy_lds_bytes();
  uint8_t* R = slab;
  load_record(R, a.states + (size_t)i * kRecordBytes);
  const uint64_t* ts = reinterpret_cast<const uint64_t*>(slab + kSlabImage);
  uint64_t w[3];
  const int n_all = legal_mask_words(R, reinterpret_cast<uint64_t*>(slab + kSlabImage), w, a.rules, slab + kSlabProbQ);
  const int n = n_all < kMaxLegal ? n_all : kMaxLegal;
  // the legal list, ascending: word order, then bit order
  int16_t* list = reinterpret_cast<int16_t*>(slab + kPolicyList);
  int base = 0;
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int word = lane + 64 * g;
    uint64_t v = word < kMaskWords ? w[g] : 0ull;
    const int c = __popcll(v);
    const int incl = wave_incl_scan(c);
    int pos = base + incl - c;
    while (v) {   // at most 244 legal moves exist; the bound only guards the buffer
      if (pos < kMaxLegal) list[pos] = (int16_t)(64 * word + __ffsll((unsigned long long)v) - 1);
      ++pos;
      v &= v - 1;
    }
    base += __shfl(incl, 63, 64);
  }
  wave_sync();
  const size_t row = (size_t)i * kMaxLegal;
  if (Q == kPList) {
    for (int k = lane; k < kMaxLegal; k += 64) a.actions[row + k] = k < n ? list[k] : (int16_t)-1;
    if (lane == 0 && a.num_legal) a.num_legal[i] = (int16_t)n;
    return;
  }
  if (Q == kPSample) {
    if (lane == 0) {
      int pick = -1;
      if (n > 0) {
        const uint4 u = philox(make_uint4(hdr_u32(R, kOffGameId), hdr_u32(R, kOffPly), hdr_u32(R, kOffEpisode), 4u),
                               a.rules.seed);
        const float* p = a.in_probs + row;
        float total = 0.0f;
        for (int k = 0; k < n; ++k) total += p[k];
        const float t = (float)(u.x >> 8) * (1.0f / 16777216.0f) * total;
        float run = 0.0f;
        for (int k = 0; k < n; ++k) {
          run += p[k];
          if (p[k] > 0.0f) pick = list[k];
          if (run > t && p[k] > 0.0f) break;
        }
      }
      a.actions[i] = (int16_t)pick;
    }
    return;
  }
  // the magnet policy: P pieces with a legal move; m moves of an action's piece
  const bool second = lane + 64 < kSquares;
  const int P = __popcll(ballot((ts[2 * lane] | ts[2 * lane + 1]) != 0)) +
                __popcll(ballot(second && (ts[2 * lane + 128] | ts[2 * lane + 129]) != 0));
  auto moves_of = [&](int x) { return __popcll(ts[2 * x]) + __popcll(ts[2 * x + 1]); };
  if (Q == kPMagnet) {
    for (int k = lane; k < kMaxLegal; k += 64)
      a.probs[row + k] = k < n ? __fdiv_rn(1.0f, (float)(P * moves_of(list[k] / 100))) : 0.0f;
    return;
  }
  // kPSearch: pi proportional to exp((q + alpha log rho + beta log pi_theta) / (alpha + beta))
  float sc[kMaxLegal / 64];
  float top = -INFINITY;
#pragma unroll
  for (int j = 0; j < kMaxLegal / 64; ++j) {
    const int k = lane + 64 * j;
    sc[j] = -INFINITY;
    if (k < n) {
      const float log_rho = -logf((float)(P * moves_of(list[k] / 100)));
      sc[j] = (a.q[row + k] + a.alpha * log_rho + a.beta * a.logpi[row + k]) / (a.alpha + a.beta);
      top = fmaxf(top, sc[j]);
    }
  }
  top = wave_max_f(top);
  float sum = 0.0f;
#pragma unroll
  for (int j = 0; j < kMaxLegal / 64; ++j) {
    sc[j] = lane + 64 * j < n ? expf(sc[j] - top) : 0.0f;
    sum += sc[j];
  }
  sum = wave_sum_f(sum);
#pragma unroll
  for (int j = 0; j < kMaxLegal / 64; ++j) a.probs[row + lane + 64 * j] = n > 0 ? sc[j] / sum : 0.0f;
}

struct GraphEntry {
  int32_t nplies, G, S;
  const void* ptrs[9];
  hipGraphExec_t exec;
};

}  // namespace

struct stratego_ctx {
  stratego_config cfg;
  hipStream_t stream;
  hipStream_t capture_stream;
  int device;
  int num_cu;
  size_t max_lds;
  double ns_per_tick;
  uint8_t* states;
  uint8_t* backup;   // copy of the states while the autotuner runs
  int32_t* err;
  unsigned long long* ts;
  unsigned int* tickets;   // per-ply work counters of the persistent fused kernel
  hipStream_t copy_stream;   // serving: record imports beside the plies (default priority)
  int32_t* srv_dev;    // serving slot lists, 2 sets (one per iteration in flight) of 4 x N
  int32_t* srv_host;   // pinned host staging of the same lists
  int64_t steps;
  int G, S;
  std::vector<GraphEntry> graphs;
  // rollout buffer (App. B.1): H time steps of N records and step outcomes
  int64_t t;               // whole-batch plies recorded so far (the current time step)
  int32_t H;
  uint8_t* hist;           // [H][N] canonical records
  uint64_t* hist_steps;    // [H][N]
  int64_t* hist_clock;     // device copy of t
  int32_t* hist_rows;      // ring rows of the plies of one enqueue
};

namespace {

inline Rules rules_of(const stratego_ctx* c) {
  Rules r;
  r.seed = c->cfg.seed;
  r.k_battleless = c->cfg.k_battleless;
  r.max_moves = c->cfg.max_moves;
  r.auto_reset = c->cfg.auto_reset;
  r.two_square = c->cfg.two_square_rule;
  r.sampler = c->cfg.sampler;
  r.chasing = c->cfg.chasing_rule;
  r.acting_obs = c->cfg.acting_obs_only;
  return r;
}

inline int grid_for(int n, int per_block) { return (n + per_block - 1) / per_block; }

bool valid_tiling(int G, int L) {
  return (G == 1 || G == 2 || G == 4 || G == 8 || G == 16) && valid_layout(L);
}

// What a launch needs to know of its device.
struct DevLimits {
  int num_cu;
  size_t max_lds;   // dynamic LDS one workgroup may use
};

// Waves per workgroup: four when their LDS fits, else two, else one; each wave
// takes its own chunks of G games.
inline int waves_for(int G, int S, size_t max_lds) {
  (void)G;
  for (int w = 4; w > 1; w >>= 1)
    if ((size_t)w * wave_lds_bytes(S) <= max_lds) return w;
  return 1;
}

// Dynamic LDS of one fused-engine workgroup.
inline size_t lds_for(int G, int S, size_t max_lds) { return (size_t)waves_for(G, S, max_lds) * wave_lds_bytes(S); }

const void* fused_kernel(int enc, bool fast, bool nomask = false) {
  if (fast && nomask && enc == kEncNone) return reinterpret_cast<const void*>(&k_ply<kFused, kEncNone, true, true>);
  if (fast)
    return enc == 1 ? reinterpret_cast<const void*>(&k_ply<kFused, 1, true>)
         : enc == 2 ? reinterpret_cast<const void*>(&k_ply<kFused, 2, true>)
         : enc == kEncNone ? reinterpret_cast<const void*>(&k_ply<kFused, kEncNone, true>)
                    : reinterpret_cast<const void*>(&k_ply<kFused, 0, true>);
  return enc == 1 ? reinterpret_cast<const void*>(&k_ply<kFused, 1>)
       : enc == 2 ? reinterpret_cast<const void*>(&k_ply<kFused, 2>)
       : enc == kEncNone ? reinterpret_cast<const void*>(&k_ply<kFused, kEncNone>)
                  : reinterpret_cast<const void*>(&k_ply<kFused, 0>);
}

// The fused ply takes the register-board path unless a competitive-play
// rule is on.
inline bool fast_rules(const Rules& r) { return !r.two_square && !r.chasing; }

// grow: observation-free plies, where a game is short next to the loop's
// fixed costs; the tile grows up to 8 games while every wave still gets two
// or more.
int launch_ply(const DevLimits& d, hipStream_t s, int mode, PlyArgs a, int G, int S, bool persistent,
               bool grow = false) {
  // fused plies without observations take the observation-free variant,
  // whatever staging layout the encoder is tuned to
  const bool no_obs = mode == kFused && a.obs == nullptr;
  const int enc = no_obs ? kEncNone : S == kLayoutBits ? 1 : S == kLayoutBits1 ? 2 : 0;
  const int W = no_obs ? 4 : (mode == kFused) ? waves_for(G, S, d.max_lds) : 4;
  const size_t lds = (size_t)W * ply_wave_lds_bytes(enc, S);
  if (lds > d.max_lds) return STRATEGO_E_INVAL;
  const void* fn = nullptr;
  switch (mode) {
    case kFused:
      fn = fused_kernel(enc, fast_rules(a.rules), a.mask == nullptr);
      break;
    case kDoMask: fn = reinterpret_cast<const void*>(&k_ply<kDoMask, 0>); break;
    case kDoEncode:
      fn = enc == 1 ? reinterpret_cast<const void*>(&k_ply<kDoEncode, 1>)
         : enc == 2 ? reinterpret_cast<const void*>(&k_ply<kDoEncode, 2>)
                    : reinterpret_cast<const void*>(&k_ply<kDoEncode, 0>);
      break;
    case kDoStep | kStepFromInput:
      fn = reinterpret_cast<const void*>(&k_ply<kDoStep | kStepFromInput, 0>);
      break;
    default: return STRATEGO_E_INVAL;
  }
  int cap = INT_MAX;
  if (persistent) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * W, lds) != hipSuccess || per_cu <= 0)
      return STRATEGO_E_INVAL;
    cap = per_cu * d.num_cu;
  }
  int tile = (mode == kFused) ? G : 1;
  if (persistent && grow) {
    const int64_t waves = (int64_t)cap * W;
    while (tile < 8 && (int64_t)a.n >= 2 * waves * (2 * tile)) tile *= 2;
  }
  a.games_per_tile = tile;
  a.tail_from = -1;
  if (persistent && a.tickets != nullptr && tile > 1) {
    // the last (about) one game per wave is handed out as single-game tiles
    const int64_t waves = (int64_t)cap * W;
    a.tail_from = (int)(a.n > waves ? (a.n - waves) / tile : 0);
  }
  a.layout = S;
  int grid = grid_for(grid_for(a.n, tile), W);
  if (grid > cap) grid = cap;
  if (grid <= 0) return STRATEGO_OK;
  void* args[] = {&a};
  if (hipLaunchKernel(fn, dim3(grid), dim3(64 * W), args, lds, s) != hipSuccess) return STRATEGO_E_HIP;
  return hipGetLastError() == hipSuccess ? STRATEGO_OK : STRATEGO_E_HIP;
}

inline DevLimits limits_of(const stratego_ctx* c) { return DevLimits{c->num_cu, c->max_lds}; }

int launch_ply(stratego_ctx* c, hipStream_t s, int mode, PlyArgs a, int G, int S, bool persistent,
               bool grow = false) {
  return launch_ply(limits_of(c), s, mode, a, G, S, persistent, grow);
}

PlyArgs base_args(stratego_ctx* c) {
  PlyArgs a;
  std::memset(&a, 0, sizeof(a));
  a.states = c->states;
  a.n = c->cfg.num_games;
  a.total = c->cfg.num_games;
  a.err = c->err;
  a.rules = rules_of(c);
  return a;
}

// Ring rows for the next nplies recorded plies (no-op without a rollout buffer).
int enqueue_hist_clock(stratego_ctx* c, hipStream_t s, int32_t nplies) {
  if (!c->hist) return STRATEGO_OK;
  hipLaunchKernelGGL(k_hist_clock, dim3(1), dim3(256), 0, s, c->hist_clock, c->hist_rows, nplies, c->H);
  return hipGetLastError() == hipSuccess ? STRATEGO_OK : STRATEGO_E_HIP;
}

void set_hist(stratego_ctx* c, PlyArgs& a, int p) {
  if (!c->hist) return;
  a.hist = c->hist;
  a.hist_steps = c->hist_steps;
  a.hist_slot = c->hist_rows + p;
}

int enqueue_plies(stratego_ctx* c, hipStream_t s, int32_t nplies, const int32_t* slots, int32_t n,
                  uint64_t* mask, int16_t* num_legal, int16_t* actions, uint8_t* obs, int8_t* done,
                  int8_t* outcome, uint8_t* reason, int16_t* ep_len, bool timed, int G, int S,
                  bool record) {
  if (nplies > kMaxTimedPlies) return STRATEGO_E_INVAL;
  if (record) {
    int rc = enqueue_hist_clock(c, s, nplies);
    if (rc != STRATEGO_OK) return rc;
  }
  // zero the per-ply work counters (a kernel, so the step can sit in a graph)
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nplies, 256)), dim3(256), 0, s,
                     reinterpret_cast<int32_t*>(c->tickets), nplies, 0);
  if (hipGetLastError() != hipSuccess) return STRATEGO_E_HIP;
  if (timed) {
    hipLaunchKernelGGL(k_ts_init, dim3(grid_for(nplies, 256)), dim3(256), 0, s, c->ts, nplies);
    if (hipGetLastError() != hipSuccess) return STRATEGO_E_HIP;
  }
  for (int p = 0; p < nplies; ++p) {
    PlyArgs a = base_args(c);
    a.slots = slots;
    a.n = n;
    a.out_base = p * n;
    a.mask = mask;
    a.num_legal = num_legal;
    a.actions_out = actions;
    a.obs = obs;
    a.done = done;
    a.outcome = outcome;
    a.reason = reason;
    a.ep_len = ep_len;
    a.ts = timed ? c->ts + 2 * p : nullptr;
    // plies with observations hand out tiles in address order from a ticket
    // counter (11% faster than a static split: the games written at any time
    // stay adjacent); observation-free plies split statically, since there a
    // ticket's round trip waits on the wave's outstanding stores (25% faster)
    a.tickets = obs ? c->tickets + p : nullptr;
    if (record) set_hist(c, a, p);
    int rc = launch_ply(c, s, kFused, a, G, S, true, obs == nullptr);
    if (rc != STRATEGO_OK) return rc;
  }
  return STRATEGO_OK;
}

}  // namespace

extern "C" {

const char* stratego_strerror(int code) {
  switch (code) {
    case STRATEGO_OK: return "ok";
    case STRATEGO_E_INVAL: return "invalid argument";
    case STRATEGO_E_NOMEM: return "device allocation failed";
    case STRATEGO_E_HIP: return "HIP runtime error";
    case STRATEGO_E_ILLEGAL_ACTION: return "illegal action for a live game";
    case STRATEGO_E_BAD_STATE: return "malformed state record";
    case STRATEGO_E_RANGE: return "time step outside the rollout buffer's window";
    default: return "unknown error";
  }
}

static int init_context(const stratego_config* cfg, void* hip_stream, stratego_ctx** out);

int stratego_init(const stratego_config* cfg, void* hip_stream, stratego_ctx** out) {
  const int rc = init_context(cfg, hip_stream, out);
  // a failed allocation leaves its error pending in the runtime; clear it so
  // that later calls do not report it as their own
  if (rc == STRATEGO_E_NOMEM) (void)hipGetLastError();
  return rc;
}

static int init_context(const stratego_config* cfg, void* hip_stream, stratego_ctx** out) {
  if (!cfg || !out) return STRATEGO_E_INVAL;
  *out = nullptr;
  if (cfg->num_games <= 0 || cfg->k_battleless <= 0 || cfg->max_moves <= 0 ||
      cfg->max_moves > 32767 || (cfg->auto_reset != 0 && cfg->auto_reset != 1) ||
      (cfg->two_square_rule != 0 && cfg->two_square_rule != 1) ||
      (cfg->sampler != kSamplerUniform && cfg->sampler != kSamplerMagnet) ||
      (cfg->chasing_rule != 0 && cfg->chasing_rule != 1) ||
      (cfg->acting_obs_only != 0 && cfg->acting_obs_only != 1))
    return STRATEGO_E_INVAL;
  int G = cfg->games_per_wg ? cfg->games_per_wg : 1;
  int S = cfg->lds_layout ? cfg->lds_layout : kLayoutBits;
  if (!valid_tiling(G, S)) return STRATEGO_E_INVAL;
  if (cfg->history_len < 0 || cfg->history_len > kMaxHistory) return STRATEGO_E_INVAL;
  stratego_ctx* c = new (std::nothrow) stratego_ctx();
  if (!c) return STRATEGO_E_NOMEM;
  c->cfg = *cfg;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->G = G;
  c->S = S;
  c->steps = 0;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return STRATEGO_E_HIP; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) { delete c; return STRATEGO_E_HIP; }
  c->num_cu = prop.multiProcessorCount;
  c->max_lds = prop.sharedMemPerBlock;
  if (lds_for(G, S, c->max_lds) > c->max_lds) { delete c; return STRATEGO_E_INVAL; }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess || khz <= 0)
    khz = 100000;
  c->ns_per_tick = 1.0e6 / (double)khz;
  const size_t nbytes = (size_t)cfg->num_games * kRecordBytes;
  if (hipMalloc(&c->states, nbytes) != hipSuccess) { delete c; return STRATEGO_E_NOMEM; }
  if (hipMalloc(&c->backup, nbytes) != hipSuccess) {
    (void)hipFree(c->states); delete c; return STRATEGO_E_NOMEM;
  }
  if (hipMalloc(&c->err, 2 * sizeof(int32_t)) != hipSuccess) {
    (void)hipFree(c->states); (void)hipFree(c->backup); delete c; return STRATEGO_E_NOMEM;
  }
  if (hipMalloc(&c->ts, 2 * sizeof(unsigned long long) * kMaxTimedPlies) != hipSuccess) {
    (void)hipFree(c->states); (void)hipFree(c->backup); (void)hipFree(c->err); delete c;
    return STRATEGO_E_NOMEM;
  }
  if (hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(c->states); (void)hipFree(c->backup); (void)hipFree(c->err); (void)hipFree(c->ts);
    delete c;
    return STRATEGO_E_HIP;
  }
  if (hipMalloc(&c->tickets, sizeof(unsigned int) * kMaxTimedPlies) != hipSuccess) {
    c->tickets = nullptr;
    c->srv_dev = nullptr;
    c->srv_host = nullptr;
    stratego_destroy(c);
    return STRATEGO_E_NOMEM;
  }
  if (hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    c->copy_stream = nullptr;
    c->srv_dev = nullptr;
    c->srv_host = nullptr;
    stratego_destroy(c);
    return STRATEGO_E_HIP;
  }
  const size_t lists = 8 * (size_t)cfg->num_games * sizeof(int32_t);
  if (hipMalloc(&c->srv_dev, lists) != hipSuccess) {
    c->srv_dev = nullptr;
    c->srv_host = nullptr;
    stratego_destroy(c);
    return STRATEGO_E_NOMEM;
  }
  if (hipHostMalloc(&c->srv_host, lists, hipHostMallocDefault) != hipSuccess) {
    c->srv_host = nullptr;
    stratego_destroy(c);
    return STRATEGO_E_NOMEM;
  }
  if (cfg->history_len > 0) {
    c->H = cfg->history_len;
    const size_t rows = (size_t)c->H * (size_t)cfg->num_games;
    auto alloc = [](auto** p, size_t bytes) {
      if (hipMalloc(reinterpret_cast<void**>(p), bytes) == hipSuccess) return true;
      *p = nullptr;
      return false;
    };
    if (!alloc(&c->hist, rows * kRecordBytes) || !alloc(&c->hist_steps, rows * sizeof(uint64_t)) ||
        !alloc(&c->hist_clock, sizeof(int64_t)) || !alloc(&c->hist_rows, sizeof(int32_t) * kMaxTimedPlies)) {
      stratego_destroy(c);
      return STRATEGO_E_NOMEM;
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<int32_t*>(c->hist_clock), 2, 0);
  }
  // kernels whose dynamic LDS may exceed the default limit
  const void* big_lds[] = {fused_kernel(0, false), fused_kernel(1, false), fused_kernel(2, false),
                           fused_kernel(0, true), fused_kernel(1, true), fused_kernel(2, true),
                           reinterpret_cast<const void*>(&k_ply<kDoEncode, 0>),
                           reinterpret_cast<const void*>(&k_ply<kDoEncode, 1>),
                           reinterpret_cast<const void*>(&k_ply<kDoEncode, 2>)};
  for (const void* f : big_lds)
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->max_lds);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->stream, c->err, 2, INT_MAX);
  int rc = stratego_reset(c, nullptr, cfg->num_games, nullptr);
  if (rc != STRATEGO_OK) { stratego_destroy(c); return rc; }
  *out = c;
  return STRATEGO_OK;
}

int stratego_reset(stratego_ctx* c, const int32_t* slots, int32_t n, const void* states) {
  if (!c || n < 0 || n > c->cfg.num_games) return STRATEGO_E_INVAL;
  if (n == 0) return STRATEGO_OK;
  const int grid = grid_for(n, 4);
  if (states) {
    hipLaunchKernelGGL(k_import, dim3(grid), dim3(256), 4 * kSlabImage, c->stream, c->states, slots, n,
                       c->cfg.num_games, reinterpret_cast<const uint8_t*>(states), c->err);
  } else {
    hipLaunchKernelGGL(k_reset_fresh, dim3(grid), dim3(256), 4 * kSlabImage, c->stream, c->states, slots,
                       n, c->cfg.num_games, rules_of(c), c->cfg.game_id_base, c->err);
  }
  return hipGetLastError() == hipSuccess ? STRATEGO_OK : STRATEGO_E_HIP;
}

int stratego_legal_mask(stratego_ctx* c, uint64_t* mask, int16_t* num_legal) {
  if (!c || !mask) return STRATEGO_E_INVAL;
  PlyArgs a = base_args(c);
  a.mask = mask;
  a.num_legal = num_legal;
  return launch_ply(c, c->stream, kDoMask, a, 4, 6, false);
}

int stratego_sample_actions(stratego_ctx* c, const uint64_t* mask, const int16_t* num_legal,
                            int16_t* actions) {
  if (!c || !mask || !num_legal || !actions) return STRATEGO_E_INVAL;
  hipLaunchKernelGGL(k_sample, dim3(grid_for(c->cfg.num_games, 4)), dim3(256), 0, c->stream, c->states,
                     c->cfg.num_games, mask, num_legal, actions, c->cfg.seed, c->cfg.sampler);
  return hipGetLastError() == hipSuccess ? STRATEGO_OK : STRATEGO_E_HIP;
}

int stratego_step(stratego_ctx* c, const int16_t* actions, int8_t* done, int8_t* outcome,
                  uint8_t* reason, int16_t* ep_len) {
  if (!c || !actions) return STRATEGO_E_INVAL;
  PlyArgs a = base_args(c);
  a.actions_in = actions;
  a.done = done;
  a.outcome = outcome;
  a.reason = reason;
  a.ep_len = ep_len;
  int rc = enqueue_hist_clock(c, c->stream, 1);
  if (rc != STRATEGO_OK) return rc;
  set_hist(c, a, 0);
  rc = launch_ply(c, c->stream, kDoStep | kStepFromInput, a, 4, 6, false);
  if (rc != STRATEGO_OK) return rc;
  c->steps += c->cfg.num_games;
  c->t += 1;
  return STRATEGO_OK;
}

int stratego_encode_obs(stratego_ctx* c, uint8_t* obs) {
  if (!c || !obs) return STRATEGO_E_INVAL;
  PlyArgs a = base_args(c);
  a.obs = obs;
  return launch_ply(c, c->stream, kDoEncode, a, 4, kLayoutBits, false);
}

int stratego_export_states(stratego_ctx* c, void* states) {
  if (!c || !states) return STRATEGO_E_INVAL;
  return hipMemcpyAsync(states, c->states, (size_t)c->cfg.num_games * kRecordBytes,
                        hipMemcpyDeviceToDevice, c->stream) == hipSuccess
             ? STRATEGO_OK
             : STRATEGO_E_HIP;
}

int stratego_run_plies(stratego_ctx* c, int32_t nplies, uint64_t* mask, int16_t* num_legal,
                       int16_t* actions, uint8_t* obs, int8_t* done, int8_t* outcome, uint8_t* reason,
                       int16_t* ep_len, int32_t use_graph, int64_t* ply_ns) {
  if (!c || nplies < 0 || use_graph < 0 || use_graph > 2) return STRATEGO_E_INVAL;
  if (ply_ns && nplies > kMaxTimedPlies) return STRATEGO_E_INVAL;
  if (nplies == 0) return STRATEGO_OK;
  const bool timed = ply_ns != nullptr;
  const int n = c->cfg.num_games;
  if (!use_graph) {
    for (int32_t p0 = 0; p0 < nplies; p0 += kMaxTimedPlies) {
      const int32_t np = nplies - p0 < kMaxTimedPlies ? nplies - p0 : kMaxTimedPlies;
      const size_t off = (size_t)p0 * n;
      int rc = enqueue_plies(c, c->stream, np, nullptr, n, mask, num_legal, actions ? actions + off : nullptr,
                             obs, done ? done + off : nullptr, outcome ? outcome + off : nullptr,
                             reason ? reason + off : nullptr, ep_len ? ep_len + off : nullptr, timed, c->G,
                             c->S, true);
      if (rc != STRATEGO_OK) return rc;
    }
  } else {
    if (nplies > kMaxTimedPlies) return STRATEGO_E_INVAL;
    const void* key[9] = {mask, num_legal, actions, obs, done, outcome, reason, ep_len,
                          timed ? (const void*)c->ts : nullptr};
    hipGraphExec_t exec = nullptr;
    for (auto& e : c->graphs) {
      if (e.nplies == nplies && e.G == c->G && e.S == c->S && std::memcmp(e.ptrs, key, sizeof(key)) == 0) {
        exec = e.exec;
        break;
      }
    }
    if (!exec) {
      hipGraph_t graph;
      if (hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
        return STRATEGO_E_HIP;
      int rc = enqueue_plies(c, c->capture_stream, nplies, nullptr, n, mask, num_legal, actions, obs,
                             done, outcome, reason, ep_len, timed, c->G, c->S, true);
      hipError_t ec = hipStreamEndCapture(c->capture_stream, &graph);
      if (rc != STRATEGO_OK) { if (ec == hipSuccess) (void)hipGraphDestroy(graph); return rc; }
      if (ec != hipSuccess) return STRATEGO_E_HIP;
      if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return STRATEGO_E_HIP;
      }
      (void)hipGraphDestroy(graph);
      if (c->graphs.size() >= 16) {
        (void)hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
      }
      GraphEntry e;
      e.nplies = nplies;
      e.G = c->G;
      e.S = c->S;
      std::memcpy(e.ptrs, key, sizeof(key));
      e.exec = exec;
      c->graphs.push_back(e);
    }
    if (use_graph == 2)   // prepare only: the graph is built and uploaded, nothing runs
      return hipGraphUpload(exec, c->stream) == hipSuccess ? STRATEGO_OK : STRATEGO_E_HIP;
    if (hipGraphLaunch(exec, c->stream) != hipSuccess) return STRATEGO_E_HIP;
  }
  if (timed) {
    hipLaunchKernelGGL(k_ts_convert, dim3(grid_for(nplies, 256)), dim3(256), 0, c->stream, c->ts, nplies,
                       c->ns_per_tick, ply_ns);
    if (hipGetLastError() != hipSuccess) return STRATEGO_E_HIP;
  }
  c->steps += (int64_t)nplies * n;
  c->t += nplies;
  return STRATEGO_OK;
}

}  // extern "C"

namespace {

// Fused plies over caller-owned records without allocation.  Their per-ply
// work counters (and the error word the ply kernel expects) live in this
// file-scope array, of which every device holds its own copy until the
// process ends; calls that overlap on one device share it.  Host code uses
// the per-device address obtained from hipGetSymbolAddress, never the
// array's name.
constexpr int kStaticMaxPlies = STRATEGO_STATIC_MAX_PLIES;
constexpr int kStaticErr = kStaticMaxPlies;   // two int32 words after the counters

}  // namespace

static __device__ __align__(256) unsigned int scratch[kStaticMaxPlies + 64];

namespace {

struct StaticDevice {
  std::once_flag once;
  int rc;
  DevLimits lim;
  unsigned int* scratch;   // this device's copy of the array
};
constexpr int kMaxStaticDevices = 64;
StaticDevice g_static[kMaxStaticDevices];

// Once per device, with that device current: the array's address there, the
// device's limits, and the LDS attribute of the kernels that need it.
int static_device(StaticDevice** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return STRATEGO_E_HIP;
  if (dev < 0 || dev >= kMaxStaticDevices) return STRATEGO_E_INVAL;
  StaticDevice& d = g_static[dev];
  std::call_once(d.once, [&]() {
    d.rc = STRATEGO_OK;
    d.scratch = nullptr;
    void* ptr = nullptr;
    hipDeviceProp_t prop;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr ||
        hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      d.rc = STRATEGO_E_HIP;
      return;
    }
    d.scratch = reinterpret_cast<unsigned int*>(ptr);
    d.lim = DevLimits{prop.multiProcessorCount, prop.sharedMemPerBlock};
    for (int enc = 0; enc < 3; ++enc)
      for (int fast = 0; fast < 2; ++fast)
        (void)hipFuncSetAttribute(fused_kernel(enc, fast != 0), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)d.lim.max_lds);
  });
  *out = &d;
  return d.rc;
}

}  // namespace

extern "C" {

int stratego_run_plies_static(const stratego_config* cfg, void* hip_stream, void* states_dev, int32_t nplies,
                              uint64_t* mask, int16_t* num_legal, int16_t* actions, uint8_t* obs, int8_t* done,
                              int8_t* outcome, uint8_t* reason, int16_t* ep_len) {
  if (!cfg || !states_dev || nplies < 0 || nplies > kStaticMaxPlies) return STRATEGO_E_INVAL;
  if (cfg->num_games <= 0 || cfg->k_battleless <= 0 || cfg->max_moves <= 0 || cfg->max_moves > 32767 ||
      (cfg->auto_reset != 0 && cfg->auto_reset != 1) ||
      (cfg->two_square_rule != 0 && cfg->two_square_rule != 1) ||
      (cfg->sampler != kSamplerUniform && cfg->sampler != kSamplerMagnet) ||
      (cfg->chasing_rule != 0 && cfg->chasing_rule != 1) ||
      (cfg->acting_obs_only != 0 && cfg->acting_obs_only != 1) || cfg->history_len != 0)
    return STRATEGO_E_INVAL;
  const int G = cfg->games_per_wg ? cfg->games_per_wg : 1;
  const int S = cfg->lds_layout ? cfg->lds_layout : kLayoutBits;
  if (!valid_tiling(G, S)) return STRATEGO_E_INVAL;
  StaticDevice* d = nullptr;
  int rc = static_device(&d);
  if (rc != STRATEGO_OK) return rc;
  if (lds_for(G, S, d->lim.max_lds) > d->lim.max_lds) return STRATEGO_E_INVAL;
  if (nplies == 0) return STRATEGO_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const int n = cfg->num_games;
  Rules rules;
  rules.seed = cfg->seed;
  rules.k_battleless = cfg->k_battleless;
  rules.max_moves = cfg->max_moves;
  rules.auto_reset = cfg->auto_reset;
  rules.two_square = cfg->two_square_rule;
  rules.sampler = cfg->sampler;
  rules.chasing = cfg->chasing_rule;
  rules.acting_obs = cfg->acting_obs_only;
  // zero this call's work counters (a kernel rather than a memset, so that the
  // call can be captured into a graph)
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nplies, 256)), dim3(256), 0, s,
                     reinterpret_cast<int32_t*>(d->scratch), nplies, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, reinterpret_cast<int32_t*>(d->scratch + kStaticErr), 2,
                     INT_MAX);
  if (hipGetLastError() != hipSuccess) return STRATEGO_E_HIP;
  for (int p = 0; p < nplies; ++p) {
    PlyArgs a;
    std::memset(&a, 0, sizeof(a));
    a.states = reinterpret_cast<uint8_t*>(states_dev);
    a.n = n;
    a.total = n;
    a.err = reinterpret_cast<int32_t*>(d->scratch + kStaticErr);
    a.rules = rules;
    a.out_base = p * n;
    a.mask = mask;
    a.num_legal = num_legal;
    a.actions_out = actions;
    a.obs = obs;
    a.done = done;
    a.outcome = outcome;
    a.reason = reason;
    a.ep_len = ep_len;
    a.tickets = obs ? d->scratch + p : nullptr;   // as in stratego_run_plies
    rc = launch_ply(d->lim, s, kFused, a, G, S, true, obs == nullptr);
    if (rc != STRATEGO_OK) return rc;
  }
  return STRATEGO_OK;
}

int stratego_run_plies_slots(stratego_ctx* c, const int32_t* slots, int32_t nslots, int32_t nplies,
                             uint64_t* mask, int16_t* actions, uint8_t* obs, int8_t* done,
                             int8_t* outcome, uint8_t* reason, int16_t* ep_len) {
  if (!c || !slots || nslots < 0 || nslots > c->cfg.num_games || nplies < 0) return STRATEGO_E_INVAL;
  if (c->hist) return STRATEGO_E_INVAL;   // the rollout buffer indexes whole-batch plies
  if (nslots == 0 || nplies == 0) return STRATEGO_OK;
  for (int32_t p0 = 0; p0 < nplies; p0 += kMaxTimedPlies) {
    const int32_t np = nplies - p0 < kMaxTimedPlies ? nplies - p0 : kMaxTimedPlies;
    const size_t off = (size_t)p0 * nslots;
    int rc = enqueue_plies(c, c->stream, np, slots, nslots, mask, nullptr, actions ? actions + off : nullptr,
                           obs, done ? done + off : nullptr, outcome ? outcome + off : nullptr,
                           reason ? reason + off : nullptr, ep_len ? ep_len + off : nullptr, false, c->G, c->S,
                           false);
    if (rc != STRATEGO_OK) return rc;
  }
  c->steps += (int64_t)nplies * nslots;
  return STRATEGO_OK;
}

int stratego_reset_resampled(stratego_ctx* c, const void* src, int32_t nsrc, int32_t per,
                             uint32_t game_id_base) {
  if (!c || !src || nsrc <= 0 || per <= 0 || (int64_t)nsrc * per > c->cfg.num_games)
    return STRATEGO_E_INVAL;
  const int64_t waves = (int64_t)nsrc * ((per + kResamplesPerWave - 1) / kResamplesPerWave);
  if ((size_t)kResampleWaves * kResampleWaveBytes > c->max_lds) return STRATEGO_E_INVAL;
  hipLaunchKernelGGL(k_resample, dim3((unsigned)((waves + kResampleWaves - 1) / kResampleWaves)),
                     dim3(64 * kResampleWaves), kResampleWaves * kResampleWaveBytes, c->stream,
                     c->states, reinterpret_cast<const uint8_t*>(src), nsrc, per, c->cfg.seed, game_id_base,
                     c->err);
  return hipGetLastError() == hipSuccess ? STRATEGO_OK : STRATEGO_E_HIP;
}

int stratego_serve(stratego_ctx* c, const stratego_request* reqs, int32_t nreq, const void* in_states,
                   void* out_states, uint8_t* obs_out, int32_t obs_by_slot, int64_t mem_budget,
                   int32_t realtime, double backfill_wait_s, stratego_request_result* results,
                   stratego_serve_stats* stats) {
  if (!c || nreq < 0 || (nreq > 0 && (!reqs || !in_states || !out_states || !results)) ||
      !(backfill_wait_s == backfill_wait_s))
    return STRATEGO_E_INVAL;
  if (c->hist) return STRATEGO_E_INVAL;   // the rollout buffer indexes whole-batch plies
  const int N = c->cfg.num_games;
  bool any_step = false;
  int64_t total_games = 0;
  for (int r = 0; r < nreq; ++r) {
    const stratego_request& q = reqs[r];
    if ((q.kind != STRATEGO_REQ_STEP && q.kind != STRATEGO_REQ_ROLLOUT) || q.num_games < 1 ||
        q.num_games > N || q.first < 0 || q.plies < 1 || q.plies > 32767 || !(q.arrival_s >= 0.0) ||
        (q.kind == STRATEGO_REQ_STEP && q.plies != 1))
      return STRATEGO_E_INVAL;
    any_step |= q.kind == STRATEGO_REQ_STEP;
    total_games += q.num_games;
  }
  if (any_step && !obs_out) return STRATEGO_E_INVAL;
  int64_t budget = mem_budget;
  if (budget <= 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return STRATEGO_E_HIP;
    budget = (int64_t)free_b;
  }
  auto bytes_of = [&](const stratego_request& q) -> int64_t {
    return (int64_t)q.num_games *
           (kRecordBytes + (q.kind == STRATEGO_REQ_STEP ? obs_bytes_per_game(rules_of(c)) : 0));
  };
  for (int r = 0; r < nreq; ++r)
    if (bytes_of(reqs[r]) > budget) return STRATEGO_E_INVAL;   // could never be admitted

  // Everything the loop uses is allocated here, once per call.  Up to two
  // iterations are in flight: iteration k is enqueued while k - 1 runs, and
  // its host-side lists use buffer set k & 1, which iteration k - 2 (waited
  // for first) used last.  A request's slots are free again once the
  // iteration that copied its records out has completed; new requests are
  // imported only into such slots, on the copy stream, so the imports
  // overlap the plies in flight and the next iteration waits for them.
  std::vector<int> order(nreq);
  for (int r = 0; r < nreq; ++r) order[r] = r;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
  std::vector<int32_t> slot_store((size_t)total_games);   // slots of request r from seg[r]
  std::vector<int64_t> seg(nreq, 0);
  std::vector<char> is_admitted(nreq, 0);
  std::vector<int32_t> remaining(nreq, 0), adm_off(nreq, 0), run_off(nreq, 0);
  std::vector<int> active, admitted, finishing[2];
  active.reserve(nreq);
  admitted.reserve(nreq);
  finishing[0].reserve(nreq);
  finishing[1].reserve(nreq);
  std::vector<int32_t> free_now, pend_free[2];
  free_now.reserve(N);
  pend_free[0].reserve(N);
  pend_free[1].reserve(N);
  for (int i = 0; i < N; ++i) free_now.push_back(N - 1 - i);
  int32_t* srv_host_dev = nullptr;
  if (hipHostGetDevicePointer((void**)&srv_host_dev, c->srv_host, 0) != hipSuccess) return STRATEGO_E_HIP;
  int32_t *h_adm[2], *h_run[2], *d_adm[2], *d_run[2];
  for (int b = 0; b < 2; ++b) {
    int32_t* hb = c->srv_host + (size_t)b * 4 * N;
    int32_t* db = c->srv_dev + (size_t)b * 4 * N;
    // admitted slots (N), then the iteration's lists packed in one run (up to 2 N)
    h_adm[b] = hb; h_run[b] = hb + N;
    d_adm[b] = db; d_run[b] = db + N;
  }
  hipEvent_t ev_ref = nullptr, ev_first = nullptr, ev_start[2] = {}, ev_end[2] = {}, ev_import[2] = {};
  bool ev_ok = hipEventCreate(&ev_ref) == hipSuccess && hipEventCreate(&ev_first) == hipSuccess;
  for (int b = 0; b < 2; ++b)
    ev_ok = ev_ok && hipEventCreate(&ev_start[b]) == hipSuccess && hipEventCreate(&ev_end[b]) == hipSuccess &&
            hipEventCreateWithFlags(&ev_import[b], hipEventDisableTiming) == hipSuccess;
  auto destroy_events = [&]() {
    for (hipEvent_t e : {ev_ref, ev_first, ev_start[0], ev_start[1], ev_end[0], ev_end[1], ev_import[0], ev_import[1]})
      if (e) (void)hipEventDestroy(e);
  };
  if (!ev_ok) { destroy_events(); return STRATEGO_E_HIP; }

  const uint8_t* in = reinterpret_cast<const uint8_t*>(in_states);
  uint8_t* out = reinterpret_cast<uint8_t*>(out_states);
  int64_t reserved = 0, game_steps = 0, peak_reserved = 0, seg_next = 0;
  int next = 0, completed = 0, iterations = 0, peak_active = 0, active_games = 0, inflight = 0;
  int64_t k = 0;
  double busy_ms = 0.0, last_end_ms = 0.0, first_ms = 0.0;
  const auto t0 = std::chrono::steady_clock::now();
  auto now_s = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  // device time reference: completion times are the iterations' end events
  // on the device clock, placed on the host clock by this event
  if (hipEventRecord(ev_ref, c->stream) != hipSuccess || hipEventSynchronize(ev_ref) != hipSuccess) {
    destroy_events();
    return STRATEGO_E_HIP;
  }
  const double t_ref = now_s();
  int rc = STRATEGO_OK;
  // wait for the oldest iteration in flight and settle its requests
  auto retire = [&]() {
    const int b = (int)((k - inflight) & 1);
    if (hipEventSynchronize(ev_end[b]) != hipSuccess) { rc = STRATEGO_E_HIP; return; }
    float ms_busy = 0.f, ms_end = 0.f;
    (void)hipEventElapsedTime(&ms_busy, ev_start[b], ev_end[b]);
    (void)hipEventElapsedTime(&ms_end, ev_ref, ev_end[b]);
    busy_ms += ms_busy;
    last_end_ms = ms_end;
    const double t_done = t_ref + ms_end / 1e3;
    for (int r : finishing[b]) results[r].done_s = t_done;
    completed += (int)finishing[b].size();
    finishing[b].clear();
    for (int32_t sl : pend_free[b]) free_now.push_back(sl);
    pend_free[b].clear();
    --inflight;
  };
  while (rc == STRATEGO_OK && completed < nreq) {
    const int b = (int)(k & 1);
    if (inflight == 2) { retire(); if (rc != STRATEGO_OK) break; }
    // 1. admit arrived requests in arrival order while free slots and the
    //    memory budget allow.  One that does not fit lets later ones that do
    //    go ahead (backfilling) until it has waited backfill_wait_s; from
    //    then on it holds its place, so that it is admitted as soon as enough
    //    slots have freed.  (backfill_wait_s < 0: strict arrival order.)
    const double t = now_s();
    int nadm = 0;
    admitted.clear();
    for (int j = next; j < nreq; ++j) {
      const int r = order[j];
      if (is_admitted[r]) continue;
      const stratego_request& q = reqs[r];
      if (realtime && q.arrival_s > t) break;
      if ((int)free_now.size() < q.num_games || reserved + bytes_of(q) > budget) {
        const double waited = t - (realtime ? q.arrival_s : 0.0);
        if (backfill_wait_s < 0.0 || waited > backfill_wait_s) break;
        continue;
      }
      is_admitted[r] = 1;
      seg[r] = seg_next;
      seg_next += q.num_games;
      adm_off[r] = nadm;
      for (int j = 0; j < q.num_games; ++j) {
        const int32_t sl = free_now.back();
        free_now.pop_back();
        slot_store[(size_t)seg[r] + j] = sl;
        h_adm[b][nadm + j] = sl;
      }
      nadm += q.num_games;
      reserved += bytes_of(q);
      active_games += q.num_games;
      remaining[r] = q.plies;
      results[r].admit_s = t;
      active.push_back(r);
      admitted.push_back(r);
    }
    while (next < nreq && is_admitted[order[next]]) ++next;   // first request not yet admitted
    peak_reserved = std::max(peak_reserved, reserved);
    peak_active = std::max(peak_active, active_games);
    if (active.empty()) {
      if (inflight > 0) { retire(); continue; }   // completions free slots
      if (next < nreq) {                           // idle until the next arrival
        const double wait = reqs[order[next]].arrival_s - now_s();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 2e-4)));
        continue;
      }
      break;
    }
    // 2. imports of the admitted records, beside the iterations in flight
    if (nadm > 0) {
      if (hipMemcpyAsync(d_adm[b], h_adm[b], nadm * sizeof(int32_t), hipMemcpyHostToDevice, c->copy_stream) !=
          hipSuccess) { rc = STRATEGO_E_HIP; break; }
      for (int r : admitted) {
        const stratego_request& q = reqs[r];
        hipLaunchKernelGGL(k_import, dim3(grid_for(q.num_games, 4)), dim3(256), 4 * kSlabImage, c->copy_stream,
                           c->states, d_adm[b] + adm_off[r], q.num_games, N, in + (size_t)q.first * kRecordBytes,
                           c->err);
      }
      if (hipEventRecord(ev_import[b], c->copy_stream) != hipSuccess ||
          hipStreamWaitEvent(c->stream, ev_import[b], 0) != hipSuccess) { rc = STRATEGO_E_HIP; break; }
    }
    // 3. one fused ply for every active game: step requests with
    //    observations, rollout requests without
    int nstep = 0, nroll = 0;
    for (int r : active) (reqs[r].kind == STRATEGO_REQ_STEP ? nstep : nroll) += reqs[r].num_games;
    // one run: step slots, their output rows, then rollout slots, copied by a
    // kernel on this stream (a copy-engine transfer ahead of every iteration
    // left the GPU idle about a fifth of the time at saturation)
    int32_t* hs = h_run[b];
    int32_t *ho = hs + nstep, *hr = hs + 2 * nstep;
    int32_t* ds = d_run[b];
    int32_t *d_rows = ds + nstep, *d_rl = ds + 2 * nstep;
    {
      int is = 0, ir = 0;
      for (int r : active) {
        const stratego_request& q = reqs[r];
        const int32_t* sl = slot_store.data() + seg[r];
        if (q.kind == STRATEGO_REQ_STEP) {
          run_off[r] = is;
          for (int j = 0; j < q.num_games; ++j) {
            hs[is + j] = sl[j];
            ho[is + j] = obs_by_slot ? sl[j] : q.first + j;
          }
          is += q.num_games;
        } else {
          run_off[r] = ir;
          for (int j = 0; j < q.num_games; ++j) hr[ir + j] = sl[j];
          ir += q.num_games;
        }
      }
    }
    {
      const int cnt = 2 * nstep + nroll;
      hipLaunchKernelGGL(k_copy_i32, dim3((cnt + 255) / 256), dim3(256), 0, c->stream, ds,
                         srv_host_dev + (hs - c->srv_host), cnt);
    }
    if (hipEventRecord(ev_start[b], c->stream) != hipSuccess) { rc = STRATEGO_E_HIP; break; }
    if (iterations == 0 && hipEventRecord(ev_first, c->stream) != hipSuccess) { rc = STRATEGO_E_HIP; break; }
    if (nstep > 0) {
      PlyArgs a = base_args(c);
      a.slots = ds;
      a.n = nstep;
      a.out_index = d_rows;
      a.obs = obs_out;
      rc = launch_ply(c, c->stream, kFused, a, c->G, c->S, true);
      if (rc != STRATEGO_OK) break;
    }
    if (nroll > 0) {
      PlyArgs a = base_args(c);
      a.slots = d_rl;
      a.n = nroll;
      rc = launch_ply(c, c->stream, kFused, a, c->G, c->S, true);
      if (rc != STRATEGO_OK) break;
    }
    game_steps += nstep + nroll;
    // 4. requests whose last ply this is: copy their records out; their
    //    slots are free once this iteration has completed
    size_t keep = 0;
    for (size_t ai = 0; ai < active.size(); ++ai) {
      const int r = active[ai];
      if (--remaining[r] > 0) { active[keep++] = r; continue; }
      const stratego_request& q = reqs[r];
      const int32_t* list = (q.kind == STRATEGO_REQ_STEP ? ds : d_rl) + run_off[r];
      hipLaunchKernelGGL(k_gather, dim3(grid_for(q.num_games, 4)), dim3(256), 0, c->stream, c->states, list,
                         q.num_games, out + (size_t)q.first * kRecordBytes);
      finishing[b].push_back(r);
      for (int j = 0; j < q.num_games; ++j) pend_free[b].push_back(slot_store[(size_t)seg[r] + j]);
      reserved -= bytes_of(q);
      active_games -= q.num_games;
    }
    active.resize(keep);
    if (hipGetLastError() != hipSuccess || hipEventRecord(ev_end[b], c->stream) != hipSuccess) {
      rc = STRATEGO_E_HIP;
      break;
    }
    ++inflight;
    ++iterations;
    ++k;
  }
  while (inflight > 0 && rc == STRATEGO_OK) retire();
  if (rc == STRATEGO_OK && iterations > 0) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev_ref, ev_first);
    first_ms = ms;
  }
  if (rc != STRATEGO_OK) (void)hipStreamSynchronize(c->stream);
  (void)hipStreamSynchronize(c->copy_stream);
  destroy_events();
  if (rc != STRATEGO_OK) return rc;
  c->steps += game_steps;
  if (stats) {
    stats->wall_s = now_s();
    stats->game_steps = game_steps;
    stats->iterations = iterations;
    stats->peak_active_games = peak_active;
    stats->peak_reserved_bytes = peak_reserved;
    stats->budget_bytes = budget;
    stats->gpu_busy_s = busy_ms / 1e3;
    stats->gpu_span_s = iterations > 0 ? (last_end_ms - first_ms) / 1e3 : 0.0;
  }
  return STRATEGO_OK;
}

int stratego_get_tiling(stratego_ctx* c, int32_t* G, int32_t* S) {
  if (!c) return STRATEGO_E_INVAL;
  if (G) *G = c->G;
  if (S) *S = c->S;
  return STRATEGO_OK;
}

int stratego_set_tiling(stratego_ctx* c, int32_t G, int32_t S) {
  if (!c || !valid_tiling(G, S) || lds_for(G, S, c->max_lds) > c->max_lds) return STRATEGO_E_INVAL;
  c->G = G;
  c->S = S;
  return STRATEGO_OK;
}

int stratego_autotune(stratego_ctx* c, uint8_t* obs, uint64_t* mask, int32_t plies,
                      stratego_tune_entry* report, int32_t max_entries, int32_t* n_entries) {
  if (!c || plies <= 0) return STRATEGO_E_INVAL;
  const int n = c->cfg.num_games;
  uint8_t* backup = c->backup;
  const size_t nbytes = (size_t)n * kRecordBytes;
  // the tuning plies advance the games; they are restored afterwards so that
  // results do not depend on whether tuning ran
  if (hipMemcpyAsync(backup, c->states, nbytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return STRATEGO_E_HIP;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int Gs[5] = {1, 2, 4, 8, 16};
  const int Ss[7] = {1, 2, 3, 4, 5, 6, 7};
  int best_G = c->G, best_S = c->S, count = 0;
  float best = 1e30f;
  int rc = STRATEGO_OK;
  for (int gi = 0; gi < 5 && rc == STRATEGO_OK; ++gi) {
    for (int si = 0; si < 7 && rc == STRATEGO_OK; ++si) {
      const int G = Gs[gi], S = Ss[si];
      const size_t lds = lds_for(G, S, c->max_lds);
      if (lds > c->max_lds) continue;
      int per_cu = 0;
      const void* fused = fused_kernel(S == kLayoutBits ? 1 : S == kLayoutBits1 ? 2 : 0, fast_rules(rules_of(c)));
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused, 64 * waves_for(G, S, c->max_lds), lds) !=
              hipSuccess ||
          per_cu <= 0)
        continue;
      // warm-up ply, then the timed plies
      rc = enqueue_plies(c, c->stream, 1, nullptr, n, mask, nullptr, nullptr, obs, nullptr, nullptr, nullptr,
                         nullptr, false, G, S, false);
      if (rc != STRATEGO_OK) break;
      (void)hipEventRecord(e0, c->stream);
      rc = enqueue_plies(c, c->stream, plies, nullptr, n, mask, nullptr, nullptr, obs, nullptr, nullptr,
                         nullptr, nullptr, false, G, S, false);
      (void)hipEventRecord(e1, c->stream);
      if (hipEventSynchronize(e1) != hipSuccess) { rc = STRATEGO_E_HIP; break; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const float us = 1000.f * ms / (float)plies;
      if (report && count < max_entries) {
        report[count].games_per_wg = G;
        report[count].lds_layout = S;
        report[count].us_per_ply = us;
      }
      ++count;
      if (us < best) { best = us; best_G = G; best_S = S; }
    }
  }
  (void)hipMemcpyAsync(c->states, backup, nbytes, hipMemcpyDeviceToDevice, c->stream);
  (void)hipStreamSynchronize(c->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != STRATEGO_OK) return rc;
  c->G = best_G;
  c->S = best_S;
  if (n_entries) *n_entries = report ? (count < max_entries ? count : max_entries) : 0;   // rows written
  return STRATEGO_OK;
}

int stratego_history_window(stratego_ctx* c, int64_t* oldest, int64_t* current) {
  if (!c) return STRATEGO_E_INVAL;
  if (oldest) *oldest = c->t - c->H > 0 ? c->t - c->H : 0;
  if (current) *current = c->t;
  return STRATEGO_OK;
}

}  // extern "C"

namespace {

// Arguments of a query at time step t, or E_RANGE outside the window.
int hist_args(stratego_ctx* c, int64_t t, const int32_t* games, int32_t count, HistArgs& h) {
  std::memset(&h, 0, sizeof(h));
  if (count < 0 || (!games && count > c->cfg.num_games)) return STRATEGO_E_INVAL;
  const int64_t T = c->t, oldest = T - c->H > 0 ? T - c->H : 0;
  if (t < oldest || t > T) return STRATEGO_E_RANGE;
  const int N = c->cfg.num_games;
  h.t = t;
  h.oldest = oldest;
  h.H = c->H;
  h.N = N;
  h.ring = c->hist;
  h.games = games;
  h.count = count;
  h.err = c->err;
  h.rules = rules_of(c);
  if (t == T) {
    h.src = c->states;
  } else {
    const size_t row = (size_t)(t % c->H) * (size_t)N;
    h.src = c->hist + row * kRecordBytes;
    h.steps = c->hist_steps + row;
  }
  return STRATEGO_OK;
}

int launch_hist(stratego_ctx* c, int q, HistArgs& h) {
  if (h.count == 0) return STRATEGO_OK;
  const void* fn = q == kQMask ? reinterpret_cast<const void*>(&k_hist<kQMask>)
                 : q == kQObs ? reinterpret_cast<const void*>(&k_hist<kQObs>)
                 : q == kQInfo ? reinterpret_cast<const void*>(&k_hist<kQInfo>)
                 : reinterpret_cast<const void*>(&k_hist<kQRecord>);
  void* args[] = {&h};
  if (hipLaunchKernel(fn, dim3(grid_for(h.count, 4)), dim3(256), args, 4 * hist_lds_bytes(q), c->stream) !=
      hipSuccess)
    return STRATEGO_E_HIP;
  return hipGetLastError() == hipSuccess ? STRATEGO_OK : STRATEGO_E_HIP;
}

}  // namespace

extern "C" {

int stratego_history_legal_mask(stratego_ctx* c, int64_t t, const int32_t* games, int32_t count,
                                uint64_t* mask, int16_t* num_legal) {
  if (!c) return STRATEGO_E_INVAL;
  HistArgs h;
  int rc = hist_args(c, t, games, count, h);
  if (rc != STRATEGO_OK || count == 0) return rc;
  if (!mask && !num_legal) return STRATEGO_E_INVAL;
  h.mask = mask;
  h.num_legal = num_legal;
  return launch_hist(c, kQMask, h);
}

int stratego_history_encode_obs(stratego_ctx* c, int64_t t, const int32_t* games, int32_t count,
                                uint8_t* obs) {
  if (!c) return STRATEGO_E_INVAL;
  HistArgs h;
  int rc = hist_args(c, t, games, count, h);
  if (rc != STRATEGO_OK || count == 0) return rc;
  if (!obs) return STRATEGO_E_INVAL;
  h.obs = obs;
  return launch_hist(c, kQObs, h);
}

int stratego_history_info(stratego_ctx* c, int64_t t, const int32_t* games, int32_t count,
                          const stratego_history_outputs* out) {
  if (!c) return STRATEGO_E_INVAL;
  HistArgs h;
  int rc = hist_args(c, t, games, count, h);
  if (rc != STRATEGO_OK || count == 0) return rc;
  if (!out) return STRATEGO_E_INVAL;
  h.out = *out;
  return launch_hist(c, kQInfo, h);
}

int stratego_history_export(stratego_ctx* c, int64_t t, const int32_t* games, int32_t count,
                            void* states) {
  if (!c) return STRATEGO_E_INVAL;
  HistArgs h;
  int rc = hist_args(c, t, games, count, h);
  if (rc != STRATEGO_OK || count == 0) return rc;
  if (!states) return STRATEGO_E_INVAL;
  h.records = reinterpret_cast<uint8_t*>(states);
  return launch_hist(c, kQRecord, h);
}

// BoardStrs (App. B), a debugging aid: formatted on the host from the
// records of time step t, copied out of the live states or the ring row.
int stratego_board_strings(stratego_ctx* c, int64_t t, const int32_t* games, int32_t count, char* out) {
  if (!c) return STRATEGO_E_INVAL;
  HistArgs h;
  int rc = hist_args(c, t, games, count, h);
  if (rc != STRATEGO_OK || count == 0) return rc;
  if (!out) return STRATEGO_E_INVAL;
  const int N = c->cfg.num_games;
  std::vector<int32_t> idx(count);
  if (games) {
    if (hipMemcpyAsync(idx.data(), games, sizeof(int32_t) * count, hipMemcpyDeviceToHost, c->stream) !=
        hipSuccess)
      return STRATEGO_E_HIP;
  } else {
    for (int32_t i = 0; i < count; ++i) idx[i] = i;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return STRATEGO_E_HIP;
  for (int32_t i = 0; i < count; ++i)
    if (idx[i] < 0 || idx[i] >= N) return STRATEGO_E_INVAL;
  static const char kSymbol[12] = {'S', '2', '3', '4', '5', '6', '7', '8', '9', 'M', 'F', 'B'};
  std::vector<uint8_t> rec(kRecordBytes);
  for (int32_t i = 0; i < count; ++i) {
    if (hipMemcpy(rec.data(), h.src + (size_t)idx[i] * kRecordBytes, kRecordBytes, hipMemcpyDeviceToHost) !=
        hipSuccess)
      return STRATEGO_E_HIP;
    char* o = out + (size_t)i * STRATEGO_BOARD_STRING_BYTES;
    int k = 0;
    for (int r = 9; r >= 0; --r) {
      for (int col = 0; col < 10; ++col) {
        const int v = (int8_t)rec[kOffBoard + 10 * r + col];
        if (v == kLake) { o[k++] = '~'; o[k++] = '~'; }
        else if (v < 0 || v >= kPieces) { o[k++] = '.'; o[k++] = '.'; }
        else {
          uint32_t w0;
          std::memcpy(&w0, rec.data() + kOffPieces + 16 * v, sizeof(w0));
          const int type = (int)(w0 & 15u);
          o[k++] = v < 40 ? 'r' : 'b';
          o[k++] = type < 12 ? kSymbol[type] : '?';
        }
        o[k++] = col == 9 ? '\n' : ' ';
      }
    }
    o[k] = 0;
  }
  return STRATEGO_OK;
}

}  // extern "C"

namespace {

int launch_policy(stratego_ctx* c, int q, PolicyArgs& a) {
  a.states = c->states;
  a.n = c->cfg.num_games;
  a.rules = rules_of(c);
  const void* fn = q == kPList ? reinterpret_cast<const void*>(&k_policy<kPList>)
                 : q == kPMagnet ? reinterpret_cast<const void*>(&k_policy<kPMagnet>)
                 : q == kPSearch ? reinterpret_cast<const void*>(&k_policy<kPSearch>)
                 : reinterpret_cast<const void*>(&k_policy<kPSample>);
  void* args[] = {&a};
  if (hipLaunchKernel(fn, dim3(grid_for(a.n, 4)), dim3(256), args, 4 * policy_lds_bytes(), c->stream) !=
      hipSuccess)
    return STRATEGO_E_HIP;
  return hipGetLastError() == hipSuccess ? STRATEGO_OK : STRATEGO_E_HIP;
}

}  // namespace

extern "C" {

int stratego_legal_list(stratego_ctx* c, int16_t* actions, int16_t* num_legal) {
  if (!c || !actions) return STRATEGO_E_INVAL;
  PolicyArgs a;
  std::memset(&a, 0, sizeof(a));
  a.actions = actions;
  a.num_legal = num_legal;
  return launch_policy(c, kPList, a);
}

int stratego_magnet_policy(stratego_ctx* c, float* probs) {
  if (!c || !probs) return STRATEGO_E_INVAL;
  PolicyArgs a;
  std::memset(&a, 0, sizeof(a));
  a.probs = probs;
  return launch_policy(c, kPMagnet, a);
}

int stratego_search_policy(stratego_ctx* c, const float* q, const float* logpi, float alpha, float beta,
                           float* probs) {
  if (!c || !q || !logpi || !probs || !(alpha >= 0.0f) || !(beta >= 0.0f) || !(alpha + beta > 0.0f) ||
      !std::isfinite(alpha + beta))
    return STRATEGO_E_INVAL;
  PolicyArgs a;
  std::memset(&a, 0, sizeof(a));
  a.q = q;
  a.logpi = logpi;
  a.alpha = alpha;
  a.beta = beta;
  a.probs = probs;
  return launch_policy(c, kPSearch, a);
}

int stratego_sample_policy(stratego_ctx* c, const float* probs, int16_t* actions) {
  if (!c || !probs || !actions) return STRATEGO_E_INVAL;
  PolicyArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in_probs = probs;
  a.actions = actions;
  return launch_policy(c, kPSample, a);
}

int stratego_get_error(stratego_ctx* c, int32_t* first_bad_slot) {
  if (!c) return STRATEGO_E_INVAL;
  int32_t h[2];
  if (hipMemcpyAsync(h, c->err, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return STRATEGO_E_HIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return STRATEGO_E_HIP;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->stream, c->err, 2, INT_MAX);
  int rc = STRATEGO_OK;
  int32_t slot = -1;
  if (h[0] != INT_MAX) { rc = STRATEGO_E_ILLEGAL_ACTION; slot = h[0]; }
  else if (h[1] != INT_MAX) { rc = STRATEGO_E_BAD_STATE; slot = h[1]; }
  if (first_bad_slot) *first_bad_slot = slot;
  return rc;
}

int stratego_current_step(stratego_ctx* c, int64_t* steps) {
  if (!c || !steps) return STRATEGO_E_INVAL;
  *steps = c->steps;
  return STRATEGO_OK;
}

int stratego_destroy(stratego_ctx* c) {
  if (!c) return STRATEGO_E_INVAL;
  (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->graphs) (void)hipGraphExecDestroy(e.exec);
  c->graphs.clear();
  (void)hipStreamDestroy(c->capture_stream);
  if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
  if (c->tickets) (void)hipFree(c->tickets);
  if (c->srv_dev) (void)hipFree(c->srv_dev);
  if (c->srv_host) (void)hipHostFree(c->srv_host);
  if (c->hist) (void)hipFree(c->hist);
  if (c->hist_steps) (void)hipFree(c->hist_steps);
  if (c->hist_clock) (void)hipFree(c->hist_clock);
  if (c->hist_rows) (void)hipFree(c->hist_rows);
  (void)hipFree(c->states);
  (void)hipFree(c->backup);
  (void)hipFree(c->err);
  (void)hipFree(c->ts);
  delete c;
  return STRATEGO_OK;
}

}  // extern "C"
