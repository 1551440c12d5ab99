// HIP kernels of libxg for gfx950 (MI355X): xorgens streams, one wavefront per
// stream, 64 consecutive words per wavefront step.
//
// Method (arXiv:1108.0486):
//   Section 2       x_i = x_{i-128} A  xor  x_{i-65} B,
//                   A = (I + L^15)(I + R^14), B = (I + L^12)(I + R^17), 32-bit words;
//   Section 1.5     W_k = W_{k-1} + omega,  out_k = x_k + (W_k xor (W_k >> 16))  (Eq. (1));
//   Section 2       x_k .. x_{k+C-1} depend only on words older than x_k while
//                   C <= s = 65, so one 64-lane wavefront computes 64 words per step.
//
// Register-resident ring.  Lane j of a wavefront owns word j of every 64-word
// chunk.  For the chunk starting at position p the wavefront holds
//   prev[j] = x_{p-128+j}   (chunk p-128 .. p-65)
//   cur[j]  = x_{p-64+j}    (chunk p-64  .. p-1)
// and computes x_{p+j} = A(prev[j]) xor B(x_{p+j-65}).  Here x_{p+j-65} is
// cur[j-1] for j >= 1 and prev[63] for j = 0: B(cur) is rotated up by one lane
// with a DPP wave rotate, and lane 0 takes B(prev[63]), which is lane 0 of the
// previous chunk's rotation.  The 128-word ring thus never leaves VGPRs inside
// the hot loop; each chunk costs about 14 VALU operations per lane and one
// coalesced 256-byte store.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xg_device.h"
#include "xg_normal.h"
#include "xg_internal.h"
#include "xg_launch.h"

namespace xg {
namespace {

using dev::box_muller;
using dev::box_muller_unordered;
using dev::group_add;
using dev::group_close;
using dev::lanes_rotate_up;
using dev::Moments;
using dev::wave_lds_sync;
using dev::splitmix64_at;
using dev::xcd_block;
using dev::xor3;
using dev::xor_and;

constexpr uint32_t kOmega = 0x9E3779B9u;       // odd integer nearest 2^31 (sqrt 5 - 1)
constexpr uint32_t kChunkOmega = 64u * kOmega;  // Weyl advance per chunk (mod 2^32)

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// x (I + L^12)(I + R^17): the operator applied to x_{i-s}.
__device__ __forceinline__ uint32_t op_lag_s(uint32_t v) {
  v ^= v << 12;
  return v ^ (v >> 17);
}

__device__ __forceinline__ uint32_t temper_weyl(uint32_t w) { return w ^ (w >> 16); }

struct Ring {
  uint32_t prev;   // x_{p-128+j}
  uint32_t cur;    // x_{p-64+j}
  uint32_t rprev;  // lane 0: B(x_{p-65}); other lanes: unused
};

__device__ __forceinline__ Ring ring_from(uint32_t prev, uint32_t cur) {
  Ring g;
  g.prev = prev;
  g.cur = cur;
  g.rprev = lanes_rotate_up(op_lag_s(prev));  // lane 0 <- B(prev[63]) = B(x_{p-65})
  return g;
}

// Computes the next 64 words x_p .. x_{p+63} (lane j: x_{p+j}) and advances g.
__device__ __forceinline__ uint32_t ring_step(Ring &g, bool lane0) {
  const uint32_t bc = op_lag_s(g.cur);
  const uint32_t rc = lanes_rotate_up(bc);     // lane j >= 1: B(x_{p+j-65}); lane 0: B(x_{p-1})
  const uint32_t bs = lane0 ? g.rprev : rc;    // B(x_{p+j-65}) on every lane
  // A(prev) = prev (I + L^15)(I + R^14) = t xor (t >> 14), t = prev xor (prev << 15)
  const uint32_t t = g.prev ^ (g.prev << 15);
  const uint32_t x = xor3(t, t >> 14, bs);
  g.prev = g.cur;
  g.cur = x;
  g.rprev = rc;                                // lane 0: B(x_{p-1}) = B(x_{p'-65}), p' = p + 64
  return x;
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }


// Writes the 128-word window ending `rem` words into chunk `x` (rem in 1..63),
// i.e. words [rem, rem + 128) of the concatenation prev | cur | x, as the new
// linear ring; rem == 0 writes prev | cur.
__device__ __forceinline__ void store_ring(uint32_t *st, uint32_t prev, uint32_t cur, uint32_t x,
                                           uint32_t rem, uint32_t lane) {
  uint32_t lo = prev, hi = cur;
  if (rem) {
    const int src = (int)((rem + lane) & 63u);
    const uint32_t a = (uint32_t)__shfl((int)prev, src);
    const uint32_t b = (uint32_t)__shfl((int)cur, src);
    const uint32_t c = (uint32_t)__shfl((int)x, src);
    const bool wrap = rem + lane >= 64u;
    lo = wrap ? b : a;
    hi = wrap ? c : b;
  }
  st[lane] = lo;
  st[64 + lane] = hi;
}

__device__ __forceinline__ void store_weyl_pos(uint32_t *st, uint32_t weyl, uint64_t pos,
                                               uint32_t lane) {
  if (lane == 0) {
    st[128] = weyl;
    st[129] = 0u;
    st[130] = (uint32_t)pos;
    st[131] = (uint32_t)(pos >> 32);
  }
}

__device__ __forceinline__ uint64_t load_pos(const uint32_t *st) {
  return (uint64_t)st[130] | ((uint64_t)st[131] << 32);
}

// Output word of type KIND for generator output o (FP32 as its bit pattern):
// u32 as is; f32 (o >> 8) * 2^-24, exact (a 24-bit integer times a power of two).
template <uint32_t KIND>
__device__ __forceinline__ uint32_t map_word(uint32_t o) {
  if constexpr (KIND == kU32) {
    return o;
  } else {
    return __float_as_uint((float)(o >> 8) * 0x1p-24f);
  }
}

// PACED: the store is followed by an issue gap of three wait states
// (s_nop 2).  Used only by the uint32 stream-major launch at unroll 2 with
// 4-byte stores: there, with one wavefront per SIMD and 1024 fronts 4 MB
// apart, spacing each wavefront's 256-byte stores this way took a 4 GiB
// launch from 790-815 us to 717-736 us on three boxes (interleaved A/B), as
// fast as the FP32 launch, whose three extra ALU operations per chunk space
// its stores anyway.  Longer gaps, other unrolls and the other layouts
// measured slower with it, so nothing else is paced.
//
// NT: a non-temporal store (the plain launches, whose rows start aligned);
// otherwise a plain one (the batch kernel: with dense output offsets most
// requests start inside a cache line, and plain stores let the L2 merge the
// partial lines at both ends of every wavefront's 256-byte store, where
// non-temporal ones took the ragged batch from 7.1 to 12.7 ms).
//
// Loops that unroll by UNROLL write UNROLL = 1 without the one-trip inner
// loop: LLVM's LICM promotes the store of a one-trip inner loop to the loop's
// exit, and the promoted store no longer carries the non-temporal hint.
template <bool NT, class T>
__device__ __forceinline__ void store_out(T v, T *p) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v, p);
  } else {
    *p = v;
  }
}

template <uint32_t KIND, bool PACED = false, bool NT = true>
__device__ __forceinline__ void emit_word(uint32_t *p, uint32_t o) {
  store_out<NT>(map_word<KIND>(o), p);
  if constexpr (PACED) asm volatile("s_nop 2");
}

// Dynamic LDS: one 256-word staging slot per wavefront of the block (wide stores).
extern __shared__ __align__(16) uint32_t xg_lds[];

__device__ __forceinline__ uint32_t *wave_stage() { return xg_lds + (threadIdx.x >> 6) * 256u; }


// ---------------------------------------------------------------------------
// A stream's state held by a wavefront: lane j has ring words j and 64 + j;
// the Weyl value W_{pos-1} and the position are wave-uniform.
// ---------------------------------------------------------------------------
struct StreamState {
  uint32_t prev;  // x_{pos-128+j}
  uint32_t cur;   // x_{pos-64+j}
  uint32_t weyl;  // W_{pos-1}
  uint64_t pos;
};

__device__ __forceinline__ StreamState load_state(const uint32_t *st) {
  const uint32_t lane = lane_id();
  StreamState s;
  s.prev = st[lane];
  s.cur = st[64 + lane];
  s.weyl = st[128];
  s.pos = load_pos(st);
  return s;
}

// Writes the state whose ring is the 128-word window ending `rem` words into
// chunk x (see store_ring); dst == nullptr (wave-uniform) writes nothing.
__device__ __forceinline__ void write_state(uint32_t *dst, uint32_t prev, uint32_t cur, uint32_t x,
                                            uint32_t rem, uint32_t weyl, uint64_t pos, uint32_t lane) {
  if (!dst) return;
  store_ring(dst, prev, cur, x, rem, lane);
  store_weyl_pos(dst, weyl, pos, lane);
}

// ---------------------------------------------------------------------------
// One stream's word sequence inside a wavefront: open (from a state), next
// (one 64-word chunk of outputs, lane j holding word j), close (the ragged last
// chunk, then the state write-back).
// ---------------------------------------------------------------------------
struct WordStream {
  Ring g;
  uint32_t w_start;  // W_{pos-1} at open
  uint32_t wbase;    // W_{p-1} for the next chunk at p
  uint32_t wlane;    // (j + 1) omega: W_{p+j} = W_{p-1} + (j + 1) omega
  uint64_t pos;
  uint32_t lane;
  bool lane0;
};

__device__ __forceinline__ WordStream open_from(const StreamState &st) {
  WordStream s;
  s.lane = lane_id();
  s.lane0 = s.lane == 0;
  s.g = ring_from(st.prev, st.cur);
  s.w_start = st.weyl;
  s.wbase = s.w_start;
  s.wlane = (s.lane + 1u) * kOmega;
  s.pos = st.pos;
  return s;
}

__device__ __forceinline__ WordStream open_stream(const uint32_t *st) { return open_from(load_state(st)); }

__device__ __forceinline__ uint32_t next_chunk(WordStream &s) {
  const uint32_t x = ring_step(s.g, s.lane0);
  const uint32_t w = s.wbase + s.wlane;
  s.wbase += kChunkOmega;
  return x + temper_weyl(w);
}

// Emits the last rem (< 64) words of an n-word request through `tail`
// (lane-indexed: lane j writes tail[j], j < rem) and writes the end state to
// dst (nullptr: nowhere).
template <uint32_t KIND, bool NT = true>
__device__ __forceinline__ void close_stream(uint32_t *dst, WordStream &s, uint64_t n, uint32_t rem,
                                             uint32_t *tail) {
  const uint32_t p0 = s.g.prev, c0 = s.g.cur;
  uint32_t x = 0u;
  if (rem) {
    x = ring_step(s.g, s.lane0);
    const uint32_t w = s.wbase + s.wlane;
    if (s.lane < rem) emit_word<KIND, false, NT>(tail, x + temper_weyl(w));
  }
  write_state(dst, p0, c0, x, rem, s.w_start + (uint32_t)n * kOmega, s.pos + n, s.lane);
}

// ---------------------------------------------------------------------------
// u32 / f32, stream-major: n words of one stream written at out[0 .. n).
// WIDE: while out is 16-byte aligned, four chunks (256 words) are staged in
// the wavefront's LDS slot and leave as one 16-byte store per lane (1 KB per
// store instruction instead of 256 B); the rest uses one 4-byte store per lane.
// ---------------------------------------------------------------------------
template <uint32_t KIND, int UNROLL, bool WIDE, bool PACED = false, bool NT = true>
__device__ __forceinline__ void serve_words_from(const StreamState &s0, uint64_t n, uint32_t *__restrict__ out,
                                                 uint32_t *dst) {
  WordStream s = open_from(s0);
  const uint32_t lane = s.lane;
  const uint64_t nfull = n >> 6;
  const uint32_t rem = (uint32_t)(n & 63u);
  uint64_t done = 0;  // chunks written by the wide loop
  if constexpr (WIDE) {
    static_assert(UNROLL % 4 == 0, "wide stores take groups of four chunks");
    if ((reinterpret_cast<uintptr_t>(out) & 15u) == 0) {
      uint32_t *stage = wave_stage();
      u32x4 *o4 = reinterpret_cast<u32x4 *>(out) + lane;
      const uint64_t nouter = nfull / UNROLL;
      for (uint64_t it = 0; it != nouter; ++it) {
#pragma unroll
        for (int q = 0; q < UNROLL / 4; ++q) {
#pragma unroll
          for (int u = 0; u < 4; ++u) stage[64 * u + lane] = map_word<KIND>(next_chunk(s));
          wave_lds_sync();  // the read below takes words other lanes wrote
          const u32x4 v = *reinterpret_cast<const u32x4 *>(stage + 4 * lane);
          wave_lds_sync();  // the next group's writes come after this read
          store_out<NT>(v, o4 + q * 64);
        }
        o4 += (UNROLL / 4) * 64;
      }
      done = nouter * UNROLL;
    }
  }
  uint32_t *o = out + done * 64 + lane;
  const uint64_t nrest = nfull - done;
  const uint64_t nouter = nrest / UNROLL;
  for (uint64_t it = 0; it != nouter; ++it) {
    if constexpr (UNROLL == 1) {
      emit_word<KIND, PACED, NT>(o, next_chunk(s));
    } else {
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) emit_word<KIND, PACED, NT>(o + u * 64, next_chunk(s));
    }
    o += UNROLL * 64;
  }
  const uint32_t nleft = (uint32_t)(nrest % UNROLL);
  for (uint32_t c = 0; c != nleft; ++c) {
    emit_word<KIND, PACED, NT>(o, next_chunk(s));
    o += 64;
  }
  close_stream<KIND, NT>(dst, s, n, rem, o);
}

template <uint32_t KIND, int UNROLL, bool WIDE, bool PACED = false>
__device__ __forceinline__ void serve_words(uint32_t *st, uint64_t n, uint32_t *__restrict__ out) {
  serve_words_from<KIND, UNROLL, WIDE, PACED>(load_state(st), n, out, st);
}

// ---------------------------------------------------------------------------
// u32 / f32, bulk-fill layout: chunk c (words 64c .. 64c + 63) of the k-th of
// `count` streams goes to out[(c count + k) 64 ..], so the wavefronts of a
// launch write one dense, advancing region of HBM instead of `count` fronts
// n words apart; the ragged last chunks (rem = n mod 64 words each) follow,
// packed, at out[64 (n / 64) count + k rem ..].  The values are those of the
// stream-major layout; only their places differ.
// ---------------------------------------------------------------------------
template <uint32_t KIND, int UNROLL>
__device__ __forceinline__ void serve_words_fill(uint32_t *__restrict__ st, uint64_t n, uint64_t k,
                                                 uint64_t count, uint32_t *__restrict__ out) {
  WordStream s = open_stream(st);
  const uint64_t nfull = n >> 6;
  const uint32_t rem = (uint32_t)(n & 63u);
  const uint64_t stride = count * 64;
  uint32_t *o = out + k * 64 + s.lane;
  const uint64_t nouter = nfull / UNROLL;
  for (uint64_t it = 0; it != nouter; ++it) {
    if constexpr (UNROLL == 1) {
      emit_word<KIND>(o, next_chunk(s));
    } else {
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) emit_word<KIND>(o + u * stride, next_chunk(s));
    }
    o += UNROLL * stride;
  }
  const uint32_t nleft = (uint32_t)(nfull % UNROLL);
  for (uint32_t c = 0; c != nleft; ++c) {
    emit_word<KIND>(o, next_chunk(s));
    o += stride;
  }
  close_stream<KIND>(st, s, n, rem, out + nfull * stride + k * rem + s.lane);
}

// ---------------------------------------------------------------------------
// normals: Box-Muller on consecutive output pairs of the call.
// ---------------------------------------------------------------------------
// Two ways to give each lane one pair of the 128-word block lo | hi (lo
// holds words 0..63, one per lane, hi words 64..127); pair_offset gives the
// pair's first word within the block.
//  - LDS (lane j takes words 2j and 2j + 1): four ds_bpermute reads and two
//    selects.  The fewest VALU instructions: with two or more wavefronts per
//    SIMD the VALU is the bound and the LDS latency hides (3 % faster than DPP
//    at four per SIMD).
//  - DPP (an even lane j takes words j and j + 1, an odd lane j words 63 + j
//    and 64 + j): each lane needs one word of its neighbour in the same chunk,
//    which a quad permutation (lanes 2i and 2i + 1 swap) supplies in the VALU,
//    two more instructions but no LDS round trip to wait for (12 % faster than
//    LDS at one wavefront per SIMD).
template <bool DPP>
__device__ __forceinline__ uint32_t pair_offset(uint32_t lane) {
  return DPP ? (lane & ~1u) + ((lane & 1u) << 6) : 2u * lane;
}

template <bool DPP>
__device__ __forceinline__ void gather_pair(uint32_t lo, uint32_t hi, uint32_t lane, uint32_t &e, uint32_t &o) {
  if constexpr (DPP) {
    // Bit selects, not ternaries, so that the swaps cannot be sunk into
    // lane-divergent branches where the neighbouring lanes are inactive.
    constexpr int kSwapPairs = 0xB1;  // quad_perm [1, 0, 3, 2]
    const uint32_t odd = 0u - (lane & 1u);  // all ones on odd lanes
    const uint32_t lo_sw = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, kSwapPairs, 0xF, 0xF, false);
    const uint32_t hi_sw = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, kSwapPairs, 0xF, 0xF, false);
    e = dev::select_bits(hi_sw, lo, odd);
    o = dev::select_bits(hi, lo_sw, odd);
  } else {
    const int se = (int)((2u * lane) & 63u);
    const int so = se + 1;
    const uint32_t e_lo = (uint32_t)__shfl((int)lo, se), e_hi = (uint32_t)__shfl((int)hi, se);
    const uint32_t o_lo = (uint32_t)__shfl((int)lo, so), o_hi = (uint32_t)__shfl((int)hi, so);
    const bool upper = lane >= 32u;
    e = upper ? e_hi : e_lo;
    o = upper ? o_hi : o_lo;
  }
}

// Stores (or accumulates) normals idx and idx + 1 of the call.  CHECKED
// compares them with n (blocks wholly inside n skip that).  The two adjacent
// 4-byte stores of a full pair become one 8-byte store, which needs only
// 4-byte alignment.
template <bool MOMENTS, bool CHECKED, bool NT = true>
__device__ __forceinline__ void consume_pair(uint32_t e, uint32_t o, uint64_t idx, uint64_t n,
                                             float *__restrict__ out, Moments &m) {
  float z0, z1;
  if constexpr (MOMENTS && !CHECKED) {
    box_muller_unordered(e, o, z0, z1);  // a whole pair into the sums: its order is immaterial
  } else {
    box_muller(e, o, z0, z1);
  }
  const bool has0 = !CHECKED || idx < n, has1 = !CHECKED || idx + 1 < n;
  if constexpr (MOMENTS) {
    // Into the open group (the caller closes groups); has1 implies has0.
    if (has0) group_add(m, z0, has1 ? z1 : 0.0f);
  } else {
    if (has0) store_out<NT>(z0, out + idx);
    if (has1) store_out<NT>(z1, out + idx + 1);
  }
}

// n normals of one stream; MOMENTS: reduce to (sum z, sum z^2) in sums[0..1]
// instead of storing them.  Consumes 2 ceil(n / 2) words.  DPP picks the
// pair gather (above).
template <bool MOMENTS, int UNROLL, bool DPP, bool NT = true>
__device__ __forceinline__ void serve_normals_from(const StreamState &s0, uint64_t n, float *__restrict__ out,
                                                   float *__restrict__ sums, uint32_t *dst) {
  const uint32_t lane = lane_id();
  const bool lane0 = lane == 0;
  Ring g = ring_from(s0.prev, s0.cur);
  const uint32_t w_start = s0.weyl;
  const uint64_t pos = s0.pos;
  uint32_t wbase = w_start;
  const uint32_t wlane = (lane + 1u) * kOmega;
  const uint64_t words = n + (n & 1u);
  const uint64_t nblk = words >> 7;     // 128-word blocks: 64 pairs, one per lane
  const uint32_t rw = (uint32_t)(words & 127u);
  Moments m = {0.f, 0.f, 0.f, 0.f, -0.f, -0.f};
  const uint64_t nsafe = n >> 7;        // blocks whose 128 normals are all below n
  const uint32_t poff = pair_offset<DPP>(lane);
  const uint64_t nouter = UNROLL > 1 ? nsafe / UNROLL : 0;  // UNROLL = 1: the loop after this one
  uint64_t b = 0;
  for (uint64_t it = 0; it != nouter; ++it, b += UNROLL) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const uint32_t xa = ring_step(g, lane0);
      const uint32_t oa = xa + temper_weyl(wbase + wlane);
      wbase += kChunkOmega;
      const uint32_t xb = ring_step(g, lane0);
      const uint32_t ob = xb + temper_weyl(wbase + wlane);
      wbase += kChunkOmega;
      uint32_t e, o;
      gather_pair<DPP>(oa, ob, lane, e, o);
      consume_pair<MOMENTS, false, NT>(e, o, ((b + u) << 7) + poff, n, out, m);
      if (MOMENTS && ((u & 3) == 3 || u == UNROLL - 1)) group_close(m);
    }
  }
  for (; b != nsafe; ++b) {
    const uint32_t xa = ring_step(g, lane0);
    const uint32_t oa = xa + temper_weyl(wbase + wlane);
    wbase += kChunkOmega;
    const uint32_t xb = ring_step(g, lane0);
    const uint32_t ob = xb + temper_weyl(wbase + wlane);
    wbase += kChunkOmega;
    uint32_t e, o;
    gather_pair<DPP>(oa, ob, lane, e, o);
    consume_pair<MOMENTS, false, NT>(e, o, (b << 7) + poff, n, out, m);
    if (MOMENTS) group_close(m);
  }
  for (; b != nblk; ++b) {
    const uint32_t xa = ring_step(g, lane0);
    const uint32_t oa = xa + temper_weyl(wbase + wlane);
    wbase += kChunkOmega;
    const uint32_t xb = ring_step(g, lane0);
    const uint32_t ob = xb + temper_weyl(wbase + wlane);
    wbase += kChunkOmega;
    uint32_t e, o;
    gather_pair<DPP>(oa, ob, lane, e, o);
    consume_pair<MOMENTS, true, NT>(e, o, (b << 7) + poff, n, out, m);
    if (MOMENTS) group_close(m);
  }
  // Tail: rw (even, < 128) more words.
  uint32_t p0 = g.prev, c0 = g.cur, xl = 0u, rem = 0u;
  if (rw) {
    uint32_t oa, ob = 0u;
    if (rw <= 64u) {
      p0 = g.prev;
      c0 = g.cur;
      xl = ring_step(g, lane0);
      oa = xl + temper_weyl(wbase + wlane);
      rem = rw & 63u;               // rw == 64 completes the chunk
      if (!rem) { p0 = g.prev; c0 = g.cur; }
    } else {
      const uint32_t xa = ring_step(g, lane0);
      oa = xa + temper_weyl(wbase + wlane);
      wbase += kChunkOmega;
      p0 = g.prev;
      c0 = g.cur;
      xl = ring_step(g, lane0);
      ob = xl + temper_weyl(wbase + wlane);
      rem = rw - 64u;
    }
    uint32_t e, o;
    gather_pair<DPP>(oa, ob, lane, e, o);
    if (poff < rw) consume_pair<MOMENTS, true, NT>(e, o, (nblk << 7) + poff, n, out, m);
    if (MOMENTS) group_close(m);
  }
  write_state(dst, p0, c0, xl, rem, w_start + (uint32_t)words * kOmega, pos + words, lane);
  if constexpr (MOMENTS) {
    // The lanes' compensated sums are folded and reduced across the
    // wavefront in FP64, then rounded once to FP32: the reduction then adds
    // well under one FP32 rounding to the error of the sums.
    double v1 = (double)m.s1 - (double)m.c1, v2 = (double)m.s2 - (double)m.c2;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      v1 += __shfl_xor(v1, off);
      v2 += __shfl_xor(v2, off);
    }
    if (lane == 0) {
      sums[0] = (float)v1;
      sums[1] = (float)v2;
    }
  }
}

template <bool MOMENTS, int UNROLL, bool DPP>
__device__ __forceinline__ void serve_normals(uint32_t *st, uint64_t n, float *__restrict__ out,
                                              float *__restrict__ sums) {
  serve_normals_from<MOMENTS, UNROLL, DPP>(load_state(st), n, out, sums, st);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------


// Seeds one stream per wavefront: ring and Weyl start from SplitMix64(seed + i),
// zero-ring guard, then 512 = 8 chunks of discarded steps.
__global__ __launch_bounds__(256) void k_init(uint32_t *__restrict__ state, uint64_t num_streams,
                                              uint64_t seed) {
  const uint64_t wid = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wid >= num_streams) return;
  const uint32_t lane = lane_id();
  const uint64_t s = seed + wid;
  uint32_t lo = (uint32_t)(splitmix64_at(s, lane + 1u) >> 32);    // x_{-128+j}
  uint32_t hi = (uint32_t)(splitmix64_at(s, lane + 65u) >> 32);   // x_{-64+j}
  const uint32_t w0 = (uint32_t)(splitmix64_at(s, 129u) >> 32);   // W
  const bool any = __any((lo | hi) != 0u);
  if (!any && lane == 63u) hi = 1u;                                // x_{-1} = 1
  Ring g = ring_from(lo, hi);
  const bool lane0 = lane == 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) (void)ring_step(g, lane0);
  uint32_t *st = state + wid * kStateWords;
  store_ring(st, g.prev, g.cur, 0u, 0u, lane);
  store_weyl_pos(st, w0 + 512u * kOmega, 0ull, lane);
}

// DPP (normals and moments): the pair gather without LDS.
template <uint32_t KIND, int UNROLL, bool WIDE, bool DPP = false>
__global__ __launch_bounds__(1024) void k_generate(uint32_t *__restrict__ state, uint64_t first,
                                                   uint64_t count, uint64_t n, void *__restrict__ out) {
  // Stream-major rows: each XCD takes a contiguous range of streams (measured
  // a few per cent faster than the plain order for this layout).
  const uint64_t wid = ((uint64_t)xcd_block() * blockDim.x + threadIdx.x) >> 6;
  if (wid >= count) return;
  uint32_t *st = state + (first + wid) * kStateWords;
  if constexpr (KIND == kU32 || KIND == kF32) {
    constexpr bool kPaced = KIND == kU32 && UNROLL == 2 && !WIDE;  // see emit_word
    serve_words<KIND, UNROLL, WIDE, kPaced>(st, n, reinterpret_cast<uint32_t *>(out) + wid * n);
  } else if constexpr (KIND == kNormal) {
    serve_normals<false, UNROLL, DPP>(st, n, reinterpret_cast<float *>(out) + wid * n, nullptr);
  } else {
    serve_normals<true, UNROLL, DPP>(st, n, nullptr, reinterpret_cast<float *>(out) + 2 * wid);
  }
}

// Bulk-fill layout (see serve_words_fill): uint32 / FP32 only.
template <uint32_t KIND, int UNROLL>
__global__ __launch_bounds__(1024) void k_fill(uint32_t *__restrict__ state, uint64_t first,
                                               uint64_t count, uint64_t n, uint32_t *__restrict__ out) {
  // Plain block order: consecutive blocks (streams, hence adjacent 256-byte
  // pieces of the dense output front) land on different XCDs, which spreads
  // every XCD's writes over the whole front.  Measured faster than giving
  // each XCD a contiguous range (xcd_block) for this layout.
  const uint64_t wid = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wid >= count) return;
  serve_words_fill<KIND, UNROLL>(state + (first + wid) * kStateWords, n, wid, count, out);
}

// ---------------------------------------------------------------------------
// skip: advance a stream by J words without producing them.
// ---------------------------------------------------------------------------

// By stepping: the recurrence runs J words and only the state is kept.
__device__ __forceinline__ void skip_by_stepping(uint32_t *st, uint64_t J) {
  WordStream s = open_stream(st);
  const uint64_t nfull = J >> 6;
  const uint32_t rem = (uint32_t)(J & 63u);
  for (uint64_t c = 0; c != nfull; ++c) (void)ring_step(s.g, s.lane0);
  const uint32_t p0 = s.g.prev, c0 = s.g.cur;
  uint32_t x = 0u;
  if (rem) x = ring_step(s.g, s.lane0);
  store_ring(st, p0, c0, x, rem, s.lane);
  store_weyl_pos(st, s.w_start + (uint32_t)J * kOmega, s.pos + J, s.lane);
}

// By jumping: with g = z^J mod P = sum_c z^(64 c) h_c(z) (h_c of degree < 64),
// T^J S0 = g(T) S0 is evaluated by Horner's rule in steps of 64 words,
//     S <- T^64 S  xor  h_c(T) S0,      c = 63 .. 0,
// where T^64 S is one wavefront chunk step on the state S, and
// h_c(T) S0 = xor of the windows T^i S0 (i < 64, bit i of h_c set); window i
// holds words x_{i-128} .. x_{i-1} of S0's continuation, so lane j's two words
// of it are x_{i-128+j} and x_{i-64+j}, staged once through LDS into
// registers.  word(c) returns h_c as 64 bits.  Needs the wavefront's LDS slot.
template <typename WordOf>
__device__ __forceinline__ void jump_state(StreamState &s, WordOf word, uint64_t J) {
  const uint32_t lane = lane_id();
  const bool lane0 = lane == 0;
  Ring r = ring_from(s.prev, s.cur);
  const uint32_t x0 = ring_step(r, lane0);             // x_0 .. x_63
  uint32_t *buf = wave_stage();                          // x_{-128} .. x_{63}
  buf[lane] = s.prev;
  buf[64 + lane] = s.cur;
  buf[128 + lane] = x0;
  wave_lds_sync();
  uint32_t xw[128];                                      // xw[k] = x_{k-128+j}
#pragma unroll
  for (int k = 0; k < 128; ++k) xw[k] = buf[lane + k];
  wave_lds_sync();                                       // the slot may be reused after this
  uint32_t slo = 0u, shi = 0u;
#pragma unroll 1
  for (int c = 63; c >= 0; --c) {
    if (c != 63) {
      Ring q = ring_from(slo, shi);
      const uint32_t nx = ring_step(q, lane0);
      slo = shi;
      shi = nx;
    }
    const uint64_t h = word(c);
    const uint32_t hlo = (uint32_t)h, hhi = (uint32_t)(h >> 32);
    uint32_t alo = 0u, ahi = 0u;
#pragma unroll
    for (int i = 0; i < 64; ++i) {
      const uint32_t bits = i < 32 ? hlo : hhi;
      const uint32_t m = (uint32_t)((int32_t)(bits << (31 - (i & 31))) >> 31);  // bit i of h_c, all ones or zero
      alo = xor_and(alo, xw[i], m);
      ahi = xor_and(ahi, xw[64 + i], m);
    }
    slo ^= alo;
    shi ^= ahi;
  }
  s.prev = slo;
  s.cur = shi;
  s.weyl += (uint32_t)J * kOmega;
  s.pos += J;
}

template <bool JUMP>
__global__ __launch_bounds__(256) void k_skip(uint32_t *__restrict__ state, uint64_t first, uint64_t count,
                                              uint64_t J, JumpPoly g) {
  const uint64_t wid = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wid >= count) return;
  uint32_t *st = state + (first + wid) * kStateWords;
  if constexpr (JUMP) {
    StreamState s = load_state(st);
    jump_state(s, [&](int c) { return g.w[c]; }, J);
    write_state(st, s.prev, s.cur, 0u, 0u, s.weyl, s.pos, lane_id());
  } else {
    skip_by_stepping(st, J);
  }
}

// Wavefronts that share one jump.  Four: at the 137-148 VGPRs per lane of the
// kernels below (at most 170 leave room for three wavefronts per SIMD), three
// such workgroups fit on a compute unit.
constexpr uint32_t kSegWaves = 4;
constexpr uint32_t kSegBlocksPerCu = 3;

// LDS of one workgroup jump: the window x_{-128} .. x_{63} of the stream's
// continuation, and the 64 window sums A_c (acc[128 c + j] lane j's low word,
// acc[128 c + 64 + j] its high word).
struct JumpLds {
  uint32_t win[192];
  uint32_t acc[64 * 128];
};

// jump_state's Horner evaluation split over the kSegWaves wavefronts of a
// workgroup: the window sums A_c = h_c(T) S0 do not depend on each other, so
// wavefront w computes A_c for c = w, w + kSegWaves, ... into LDS; then
// wavefront 0 runs the chain S <- T^64 S xor A_c, c = 63 .. 0, and its s holds
// T^J s on return (the others' s is unchanged).  Every thread of the
// workgroup calls it with the same s; lane c's h_lo / h_hi hold h_c (so the
// coefficients come from registers, read with v_readlane, and the masks from
// scalar bit-field extracts).  Ends with a barrier: lds may be reused at once.
__device__ __forceinline__ void jump_state_wg(StreamState &s, int h_lo, int h_hi, uint64_t J, JumpLds &lds,
                                              uint32_t wave) {
  const uint32_t lane = lane_id();
  const bool lane0 = lane == 0;
  if (wave == 0) {
    Ring r0 = ring_from(s.prev, s.cur);
    const uint32_t x0 = ring_step(r0, lane0);  // x_0 .. x_63
    lds.win[lane] = s.prev;
    lds.win[64 + lane] = s.cur;
    lds.win[128 + lane] = x0;
  }
  __syncthreads();
  uint32_t xw[128];  // xw[i] = x_{i-128+j}
#pragma unroll
  for (int i = 0; i < 128; ++i) xw[i] = lds.win[lane + i];
#pragma unroll 1
  for (uint32_t c = wave; c < 64u; c += kSegWaves) {
    const uint32_t hlo = (uint32_t)__builtin_amdgcn_readlane(h_lo, (int)c);
    const uint32_t hhi = (uint32_t)__builtin_amdgcn_readlane(h_hi, (int)c);
    uint32_t alo = 0u, ahi = 0u;
#pragma unroll
    for (int i = 0; i < 64; ++i) {
      const uint32_t bits = i < 32 ? hlo : hhi;
      const uint32_t m = (uint32_t)((int32_t)(bits << (31 - (i & 31))) >> 31);  // bit i of h_c, all ones or zero
      alo = xor_and(alo, xw[i], m);
      ahi = xor_and(ahi, xw[64 + i], m);
    }
    lds.acc[128u * c + lane] = alo;
    lds.acc[128u * c + 64u + lane] = ahi;
  }
  __syncthreads();
  if (wave == 0) {
    uint32_t slo = lds.acc[128u * 63u + lane], shi = lds.acc[128u * 63u + 64u + lane];
#pragma unroll 4
    for (int c = 62; c >= 0; --c) {
      Ring rc = ring_from(slo, shi);
      const uint32_t nx = ring_step(rc, lane0);
      slo = shi ^ lds.acc[128u * c + lane];
      shi = nx ^ lds.acc[128u * c + 64u + lane];
    }
    s.prev = slo;
    s.cur = shi;
    s.weyl += (uint32_t)J * kOmega;
    s.pos += J;
  }
  __syncthreads();  // win and acc are free again
}

// Few streams: one workgroup of kSegWaves wavefronts per stream.
__global__ __launch_bounds__(kSegWaves * 64) void k_skip_wg(uint32_t *__restrict__ state, uint64_t first, uint64_t J,
                                                            JumpPoly g) {
  __shared__ JumpLds lds;
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint32_t *st = state + (first + blockIdx.x) * kStateWords;
  StreamState s = load_state(st);
  const uint64_t h = g.w[lane_id()];  // lane c holds h_c
  jump_state_wg(s, (int)(uint32_t)h, (int)(uint32_t)(h >> 32), J, lds, wave);
  if (wave == 0) write_state(st, s.prev, s.cur, 0u, 0u, s.weyl, s.pos, lane_id());
}

// Box-Muller on caller-supplied word pairs (the same device function the
// generators use): out[2m], out[2m + 1] from words[2m], words[2m + 1].
__global__ __launch_bounds__(256) void k_box_muller(const uint32_t *__restrict__ words, uint64_t pairs,
                                                    float *__restrict__ out) {
  const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= pairs) return;
  float z0, z1;
  box_muller(words[2 * m], words[2 * m + 1], z0, z1);
  out[2 * m] = z0;
  out[2 * m + 1] = z1;
}

// Workspace words of the batch kernels: work[0] the queue counter, work[1]
// the error word, work[2] the queue items (groups), work[3] the table entries.
__global__ void k_work_init(uint32_t *work, uint32_t num_groups, uint32_t num_reqs) {
  if (threadIdx.x < 64) work[threadIdx.x] = threadIdx.x == 2 ? num_groups : threadIdx.x == 3 ? num_reqs : 0u;
}

// Re-arms the queue of a table that is already in place.
__global__ void k_work_requeue(uint32_t *work) {
  if (threadIdx.x == 0) work[0] = 0u;
}

// Checks of a segment entry (kReqSegment): tile k of a longer request, whose
// start state sits in staging slot `slot`.
__device__ __forceinline__ bool seg_entry_ok(const xg_request &q, uint64_t num_streams, const SegmentArgs &seg) {
  const uint32_t k = (q.flags >> 8) & 0xFFu, slot = q.flags >> 16;
  return (q.flags & kReqSegment) && !(q.flags & kReqUndefinedBits) && q.stream < num_streams &&
         q.dtype <= XG_NORMAL && seg.stage && slot < seg.max_slots && k <= seg.max_k && (k == 0 || seg.jump_table);
}

// Start state of every segment entry of a table: its stream's state jumped by
// k L words (k = 0: a copy) into staging slot `slot`.  One wavefront per
// entry (work[3] entries); others, and entries that fail the checks, are
// skipped (the batch kernel skips those too).  The batch kernel then starts
// each segment from its slot, so no segment reads a stream state that the
// request's last segment rewrites.
__global__ __launch_bounds__(kSegWaves * 64) void k_seg_starts(const uint32_t *__restrict__ state,
                                                               uint64_t num_streams,
                                                               const xg_request *__restrict__ reqs,
                                                               const uint32_t *__restrict__ work,
                                                               SegmentArgs seg) {
  // One workgroup per segment entry (grid-stride over the table); the jump by
  // k L words is jump_state_wg with the polynomial of table entry k - 1.
  __shared__ JumpLds lds;
  const uint32_t lane = lane_id();
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t entries = work[3];
  for (uint32_t r = blockIdx.x; r < entries; r += gridDim.x) {
    const xg_request q = reqs[r];  // the same on every thread of the workgroup
    if (!(q.flags & kReqSegment) || !seg_entry_ok(q, num_streams, seg)) continue;
    const uint32_t k = (uint32_t)__builtin_amdgcn_readfirstlane((int)((q.flags >> 8) & 0xFFu));
    const uint32_t slot = q.flags >> 16;
    StreamState s = load_state(state + q.stream * kStateWords);
    uint32_t *dst = seg.stage + (uint64_t)slot * kStateWords;
    if (k) {
      const uint64_t h = seg.jump_table[(uint64_t)(k - 1) * 64 + lane];  // lane c holds h_c
      jump_state_wg(s, (int)(uint32_t)h, (int)(uint32_t)(h >> 32), (uint64_t)k * seg.seg_words, lds, wave);
    }
    if (wave == 0) write_state(dst, s.prev, s.cur, 0u, 0u, s.weyl, s.pos, lane);
  }
}

// Persistent batched kernel (launched with no more blocks than the device
// holds at once): each wavefront serves the group of its own index, then takes
// groups from an atomic queue (work[0], counting from the grid's wavefronts)
// until it passes work[2] groups; every wavefront reaches the exit.  A plain
// entry reads and rewrites its stream's state; a segment entry
// starts from its staged start state and only the request's last segment
// writes the stream's state.  Outputs leave through plain (cached) stores
// (emit_word).
template <int UNROLL, bool WIDE>
__global__ __launch_bounds__(1024) void k_batch(uint32_t *__restrict__ state, uint64_t num_streams,
                                                const xg_request *__restrict__ reqs,
                                                const uint32_t *__restrict__ groups, uint32_t *__restrict__ out,
                                                uint64_t out_elems, uint32_t *__restrict__ work,
                                                SegmentArgs seg) {
  const uint32_t lane = lane_id();
  const uint32_t num_groups = work[2], num_reqs = work[3];
  // Items come largest first.  A wavefront takes `take` consecutive items per
  // trip to the queue: one while they are large, then as many (a power of two
  // up to kBatchMaxTake) as fit kBatchTakeWords words at the size of the items
  // it served last, so that small items do not make the one counter's atomics
  // the bound (same-address atomics complete one at a time, and 2048
  // wavefronts on items of a few thousand words ask for more than that).
  // A wavefront's first item is its own index in the grid (the first pops
  // would hand out exactly those items, one atomic at a time); later trips
  // take items from the counter, offset by the wavefronts in the grid.
  const uint32_t wpb = blockDim.x >> 6;
  const uint32_t waves = gridDim.x * wpb;
  uint32_t g0 = blockIdx.x * wpb + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint32_t take = 1;
  for (;;) {
    if (g0 >= num_groups) break;
    const uint32_t g_end = num_groups - g0 < take ? num_groups : g0 + take;
    uint64_t served = 0;
    for (uint32_t g = g0; g < g_end; ++g) {
      const uint32_t r0 = groups[g], r1 = groups[g + 1];
      if (r0 > r1 || r1 > num_reqs) {
        if (lane == 0) atomicOr(&work[1], 1u);
        continue;
      }
      for (uint32_t r = r0; r < r1; ++r) {
        const xg_request q = reqs[r];
        const bool is_seg = (q.flags & kReqSegment) != 0;
        const bool ok = (is_seg ? seg_entry_ok(q, num_streams, seg)
                                : q.stream < num_streams && q.dtype <= XG_NORMAL && q.flags == 0u) &&
                        q.out_offset <= out_elems && q.n <= out_elems - q.out_offset;
        if (!ok) {
          if (lane == 0) atomicOr(&work[1], 1u);
          continue;
        }
        uint32_t *st = state + q.stream * kStateWords;
        const uint32_t *src = is_seg ? seg.stage + (uint64_t)(q.flags >> 16) * kStateWords : st;
        uint32_t *dst = !is_seg || (q.flags & kReqLast) ? st : nullptr;
        const StreamState s0 = load_state(src);
        uint32_t *o = out + q.out_offset;
        if (q.dtype == XG_U32) {
          serve_words_from<kU32, UNROLL, WIDE, false, false>(s0, q.n, o, dst);
        } else if (q.dtype == XG_F32) {
          serve_words_from<kF32, UNROLL, WIDE, false, false>(s0, q.n, o, dst);
        } else {
          serve_normals_from<false, UNROLL, true, false>(s0, q.n, reinterpret_cast<float *>(o), nullptr, dst);
        }
        served += q.n;
      }
    }
    // the largest power of two t <= kBatchMaxTake with t such items in kBatchTakeWords
    const uint64_t budget = kBatchTakeWords * (g_end - g0);
    take = 1;
    while (take < kBatchMaxTake && served * (2u * take) <= budget) take <<= 1;
    uint32_t c = 0;
    if (lane == 0) c = atomicAdd(&work[0], take);
    g0 = waves + (uint32_t)__builtin_amdgcn_readfirstlane((int)c);
  }
}

template <uint32_t KIND>
hipError_t launch_generate_k(const Shape &sh, dim3 grid, dim3 block, uint32_t *state, uint64_t first,
                             uint64_t count, uint64_t n, void *out, int num_cus, hipStream_t stream) {
  hipError_t e = hipSuccess;
  constexpr bool kWords = KIND == kU32 || KIND == kF32;
  if constexpr (!kWords) {
    // Normals with fewer than two wavefronts per SIMD: the DPP pair gather.
    if (count < 8u * (uint64_t)(num_cus > 0 ? num_cus : 1)) {
      switch (sh.unroll) {
        case 1: return launch((k_generate<KIND, 1, false, true>), grid, block, 0, stream, state, first, count, n, out);
        case 2: return launch((k_generate<KIND, 2, false, true>), grid, block, 0, stream, state, first, count, n, out);
        case 4: return launch((k_generate<KIND, 4, false, true>), grid, block, 0, stream, state, first, count, n, out);
        default: return launch((k_generate<KIND, 8, false, true>), grid, block, 0, stream, state, first, count, n, out);
      }
    }
  }
  const bool wide = kWords && sh.store_words == 4;
  const size_t lds = wide ? (size_t)sh.waves_per_block * 1024u : 0u;
  if (wide) {
    if (sh.unroll == 4) {
      e = launch((k_generate<KIND, 4, kWords>), grid, block, lds, stream, state, first, count, n, out);
    } else {
      e = launch((k_generate<KIND, 8, kWords>), grid, block, lds, stream, state, first, count, n, out);
    }
    return e;
  }
  switch (sh.unroll) {
    case 1: e = launch((k_generate<KIND, 1, false>), grid, block, 0, stream, state, first, count, n, out); break;
    case 2: e = launch((k_generate<KIND, 2, false>), grid, block, 0, stream, state, first, count, n, out); break;
    case 4: e = launch((k_generate<KIND, 4, false>), grid, block, 0, stream, state, first, count, n, out); break;
    default: e = launch((k_generate<KIND, 8, false>), grid, block, 0, stream, state, first, count, n, out); break;
  }
  return e;
}

}  // namespace

uint32_t auto_waves_per_block(uint64_t count, int num_cus) {
  const uint64_t cus = num_cus > 0 ? (uint64_t)num_cus : 1;
  if (count >= 4 * cus) return 4;
  if (count >= 2 * cus) return 2;
  return 1;
}

bool shape_valid(const Shape &s) {
  const bool wpb = s.waves_per_block == 1 || s.waves_per_block == 2 || s.waves_per_block == 4 ||
                   s.waves_per_block == 8 || s.waves_per_block == 16;
  const bool un = s.unroll == 1 || s.unroll == 2 || s.unroll == 4 || s.unroll == 8;
  const bool sw = s.store_words == 1 || (s.store_words == 4 && s.unroll >= 4);
  return wpb && un && sw && s.blocks_per_cu >= 1 && s.blocks_per_cu <= 32;
}

hipError_t launch_init(uint32_t *state, uint64_t num_streams, uint64_t seed, hipStream_t stream) {
  hipError_t e = hipSuccess;
  const uint64_t blocks = (num_streams + 3) / 4;
  e = launch(k_init, dim3((uint32_t)blocks), dim3(256), 0, stream, state, num_streams, seed);
  return e;
}

hipError_t launch_fill(Kind kind, const Shape &shape, uint32_t *state, uint64_t first, uint64_t count,
                       uint64_t n, uint32_t *out, hipStream_t stream) {
  hipError_t e = hipSuccess;
  const uint64_t wpb = shape.waves_per_block;
  const dim3 grid((uint32_t)((count + wpb - 1) / wpb));
  const dim3 block((uint32_t)(wpb * kWave));
  const bool f = kind == kF32;
  switch (shape.unroll) {
    case 1: if (f) e = launch((k_fill<kF32, 1>), grid, block, 0, stream, state, first, count, n, out);
            else e = launch((k_fill<kU32, 1>), grid, block, 0, stream, state, first, count, n, out);
            break;
    case 2: if (f) e = launch((k_fill<kF32, 2>), grid, block, 0, stream, state, first, count, n, out);
            else e = launch((k_fill<kU32, 2>), grid, block, 0, stream, state, first, count, n, out);
            break;
    case 4: if (f) e = launch((k_fill<kF32, 4>), grid, block, 0, stream, state, first, count, n, out);
            else e = launch((k_fill<kU32, 4>), grid, block, 0, stream, state, first, count, n, out);
            break;
    default: if (f) e = launch((k_fill<kF32, 8>), grid, block, 0, stream, state, first, count, n, out);
             else e = launch((k_fill<kU32, 8>), grid, block, 0, stream, state, first, count, n, out);
             break;
  }
  return e;
}

hipError_t launch_box_muller(const uint32_t *words, uint64_t pairs, float *out, hipStream_t stream) {
  hipError_t e = hipSuccess;
  e = launch(k_box_muller, dim3((uint32_t)((pairs + 255) / 256)), dim3(256), 0, stream, words, pairs, out);
  return e;
}

hipError_t launch_skip(uint32_t *state, uint64_t first, uint64_t count, uint64_t J, const JumpPoly *g,
                       int num_cus, hipStream_t stream) {
  hipError_t e = hipSuccess;
  const dim3 grid((uint32_t)((count + 3) / 4)), block(256);
  if (g && count <= (uint64_t)(num_cus > 0 ? num_cus : 1) * kSegBlocksPerCu) {
    // Streams that all fit on the chip at once as workgroup jumps: each jump
    // takes about a quarter of one wavefront's time.
    e = launch(k_skip_wg, dim3((uint32_t)count), dim3(kSegWaves * 64), 0, stream, state, first, J, *g);
  } else if (g) {
    e = launch((k_skip<true>), grid, block, 4 * 1024, stream, state, first, count, J, *g);
  } else {
    JumpPoly none;
    for (int i = 0; i < 64; ++i) none.w[i] = 0;
    e = launch((k_skip<false>), grid, block, 0, stream, state, first, count, J, none);
  }
  return e;
}

hipError_t launch_generate(Kind kind, const Shape &shape, uint32_t *state, uint64_t first,
                           uint64_t count, uint64_t n, void *out, int num_cus, hipStream_t stream) {
  const uint64_t wpb = shape.waves_per_block;
  const dim3 grid((uint32_t)((count + wpb - 1) / wpb));
  const dim3 block((uint32_t)(wpb * kWave));
  switch (kind) {
    case kU32: return launch_generate_k<kU32>(shape, grid, block, state, first, count, n, out, num_cus, stream);
    case kF32: return launch_generate_k<kF32>(shape, grid, block, state, first, count, n, out, num_cus, stream);
    case kNormal:
      return launch_generate_k<kNormal>(shape, grid, block, state, first, count, n, out, num_cus, stream);
    default: return launch_generate_k<kMoments>(shape, grid, block, state, first, count, n, out, num_cus, stream);
  }
}

hipError_t launch_work_init(uint32_t *work, uint32_t num_groups, uint32_t num_reqs, hipStream_t stream) {
  return launch(k_work_init, dim3(1), dim3(64), 0, stream, work, num_groups, num_reqs);
}

hipError_t launch_work_requeue(uint32_t *work, hipStream_t stream) {
  return launch(k_work_requeue, dim3(1), dim3(64), 0, stream, work);
}

hipError_t launch_seg_starts(const uint32_t *state, uint64_t num_streams, const xg_request *reqs,
                             uint32_t max_entries, const uint32_t *work, const SegmentArgs &seg, int num_cus,
                             hipStream_t stream) {
  if (max_entries == 0) return hipSuccess;
  // As many workgroups as fit on the chip at once, each taking every
  // gridDim-th entry.
  const uint32_t slots = (num_cus > 0 ? (uint32_t)num_cus : 1u) * kSegBlocksPerCu;
  const uint32_t blocks = max_entries < slots ? max_entries : slots;
  return launch(k_seg_starts, dim3(blocks), dim3(kSegWaves * 64), 0, stream, state, num_streams, reqs, work, seg);
}

hipError_t launch_batch(const Shape &shape, int num_cus, uint32_t *state, uint64_t num_streams,
                        const xg_request *reqs, const uint32_t *groups, uint32_t max_groups, uint32_t *out,
                        uint64_t out_elems, uint32_t *work, hipStream_t stream, const SegmentArgs *seg) {
  uint64_t blocks = (uint64_t)(num_cus > 0 ? num_cus : 1) * shape.blocks_per_cu;
  const uint64_t need = ((uint64_t)max_groups + shape.waves_per_block - 1) / shape.waves_per_block;
  if (need < blocks) blocks = need ? need : 1;
  const dim3 block(shape.waves_per_block * kWave);
  const size_t lds = shape.store_words == 4 ? (size_t)shape.waves_per_block * 1024u : 0u;  // wide-store staging
  SegmentArgs sa{};
  if (seg) sa = *seg;
  auto run = [&](auto kernel) {
    return launch_persistent(kernel, blocks, block, lds, num_cus, stream, state, num_streams, reqs, groups, out,
                             out_elems, work, sa);
  };
  if (shape.store_words == 4) return shape.unroll == 4 ? run(k_batch<4, true>) : run(k_batch<8, true>);
  switch (shape.unroll) {
    case 1: return run(k_batch<1, false>);
    case 2: return run(k_batch<2, false>);
    case 4: return run(k_batch<4, false>);
    default: return run(k_batch<8, false>);
  }
}

}  // namespace xg
