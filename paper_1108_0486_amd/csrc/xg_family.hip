// HIP kernels of libxg for two further xorgens members, both with r = 64 and
// s = 33 (Section 2: s = r/2 + 1, gcd(r, s) = 1; Section 1.5: period
// 2^n - 1 for n = r w a power of two up to 4096):
//   n2048: w = 32, (a, b, c, d) = (19, 19,  9, 18), gamma = 16;
//   w64:   w = 64, (a, b, c, d) = (24, 22, 37, 45), gamma = 32;
// with x_i = x_{i-64} (I + L^a)(I + R^b) xor x_{i-33} (I + L^c)(I + R^d), the
// Weyl sequence W_k = W_{k-1} + omega (omega the odd integer nearest
// 2^{w-1}(sqrt 5 - 1)) and out_k = x_k + (W_k xor (W_k >> gamma)) mod 2^w
// (Eq. (1)).  The paper gives no shifts for these members; each quadruple
// makes the characteristic polynomial primitive of degree n.
//
// Parallel step: x_p .. x_{p+31} depend only on words older than x_p while
// 32 <= s, so a step computes 32 words of a stream.  A 64-lane wavefront runs
// two streams with interleaved lanes: lane 2j + h holds word j of stream h
// (h = 0, 1), so every lane works and a step writes 64 words.  For the chunk
// at p, lane 2j + h holds
//   prev = x_{p-64+j},  cur = x_{p-32+j}          (of stream h)
// and x_{p+j} = A(prev) xor B(x_{p+j-33}), where x_{p+j-33} is cur[j-1] for
// j >= 1 and prev[31] for j = 0.  Rotating B(cur) up by two lanes moves word
// j - 1 of each stream to word j of the same stream; lanes 0 and 1 receive
// word 31 of their own stream, which is B(prev[31]) one step later, so they
// keep the previous step's rotation (as the one-stream kernel does on lane 0).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "xg_device.h"
#include "xg_normal.h"
#include "xg_internal.h"
#include "xg_launch.h"
#include "xg_fam_batch.h"

namespace xg {
namespace {

struct MemberN2048 {
  using word = uint32_t;
  static constexpr uint32_t a = 19, b = 19, c = 9, d = 18, gamma = 16;
  static constexpr word omega = 0x9E3779B9u;
  // ring u32[64] | W | reserved | pos u64
  static constexpr uint32_t state_bytes = 272, weyl_off = 256, pos_off = 264;
};

struct MemberW64 {
  using word = uint64_t;
  static constexpr uint32_t a = 24, b = 22, c = 37, d = 45, gamma = 32;
  static constexpr word omega = 0x9E3779B97F4A7C15ull;
  // ring u64[64] | W | pos
  static constexpr uint32_t state_bytes = 528, weyl_off = 512, pos_off = 520;
};

constexpr uint32_t kStep = 32;  // words of one stream per wavefront step

using dev::splitmix64_at;
using dev::xcd_block;

// Lane l receives lane l-2's value (mod 64): two one-lane rotations.
__device__ __forceinline__ uint32_t rot2(uint32_t v) { return dev::lanes_rotate_up(dev::lanes_rotate_up(v)); }
__device__ __forceinline__ uint64_t rot2(uint64_t v) {
  return (uint64_t)rot2((uint32_t)v) | ((uint64_t)rot2((uint32_t)(v >> 32)) << 32);
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return dev::xor3(a, b, c); }
__device__ __forceinline__ uint64_t xor3(uint64_t a, uint64_t b, uint64_t c) {
  return (uint64_t)dev::xor3((uint32_t)a, (uint32_t)b, (uint32_t)c) |
         ((uint64_t)dev::xor3((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32)) << 32);
}

__device__ __forceinline__ uint32_t shfl_word(uint32_t v, int src) { return (uint32_t)__shfl((int)v, src); }
__device__ __forceinline__ uint64_t shfl_word(uint64_t v, int src) {
  return (uint64_t)(uint32_t)__shfl((int)(uint32_t)v, src) |
         ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(v >> 32), src) << 32);
}

template <class M>
__device__ __forceinline__ typename M::word op_b(typename M::word v) {
  v ^= v << M::c;
  return v ^ (v >> M::d);
}

template <class M>
struct Ring2 {
  using word = typename M::word;
  word prev, cur, rprev;

  __device__ __forceinline__ void open(word p, word c) {
    prev = p;
    cur = c;
    rprev = rot2(op_b<M>(p));  // word 0: B(prev[31]) = B(x_{p-33})
  }

  // x_{p+j} on lane 2j + h; advances the ring by one chunk.
  __device__ __forceinline__ word step(bool word0) {
    const word bc = op_b<M>(cur);
    const word rc = rot2(bc);              // word j >= 1: B(x_{p+j-33}); word 0: B(x_{p-1})
    const word bs = word0 ? rprev : rc;
    const word t = prev ^ (prev << M::a);  // prev (I + L^a) (I + R^b) = t xor (t >> b)
    const word x = xor3(t, t >> M::b, bs);
    prev = cur;
    cur = x;
    rprev = rc;                            // word 0: B(x_{p-1}) = B(x_{p'-33}), p' = p + 32
    return x;
  }
};

// Output word of KIND for generator output o, as stored (FP as bit pattern).
//   w = 32: u32 o; f32 (o >> 8) 2^-24.   w = 64: u64 o; f64 (o >> 11) 2^-53.
// Both FP maps are exact (an integer of at most 24 / 53 bits times a power of 2).
template <class M, uint32_t KIND>
__device__ __forceinline__ typename M::word map_out(typename M::word o) {
  if constexpr (sizeof(typename M::word) == 4) {
    if constexpr (KIND == kU32) return o;
    else return __float_as_uint((float)(o >> 8) * 0x1p-24f);
  } else {
    if constexpr (KIND == kU64) return o;
    else return (uint64_t)__double_as_longlong((double)(o >> 11) * 0x1p-53);
  }
}

template <class M>
__device__ __forceinline__ typename M::word seed_word(uint64_t v) {
  if constexpr (sizeof(typename M::word) == 4) return (uint32_t)(v >> 32);  // the high w bits
  else return v;
}

struct Lanes {
  uint32_t lane, h, j;
  uint64_t k;    // stream index within the launch
  bool active;   // k < count
};

__device__ __forceinline__ Lanes lanes_of(uint64_t count, uint32_t block) {
  Lanes L;
  L.lane = threadIdx.x & 63u;
  L.h = L.lane & 1u;
  L.j = L.lane >> 1;
  const uint64_t pair = ((uint64_t)block * blockDim.x + threadIdx.x) >> 6;
  L.k = 2 * pair + L.h;
  L.active = L.k < count;
  return L;
}

// Writes the 64-word window that ends `rem` words into chunk x (rem in 0..31)
// as stream h's new linear ring, then W and pos.
template <class M>
__device__ __forceinline__ void store_state(unsigned char *st, const Lanes &L, typename M::word prev,
                                            typename M::word cur, typename M::word x, uint32_t rem,
                                            typename M::word weyl, uint64_t pos) {
  using word = typename M::word;
  word lo = prev, hi = cur;
  if (rem) {  // wave-uniform
    const uint32_t js = (rem + L.j) & 31u;
    const int src = (int)(2 * js + L.h);
    const word a = shfl_word(prev, src), b = shfl_word(cur, src), c = shfl_word(x, src);
    const bool wrap = rem + L.j >= 32u;
    lo = wrap ? b : a;
    hi = wrap ? c : b;
  }
  if (!L.active) return;
  word *ring = reinterpret_cast<word *>(st);
  ring[L.j] = lo;
  ring[32 + L.j] = hi;
  if (L.j == 0) {
    *reinterpret_cast<word *>(st + M::weyl_off) = weyl;
    if constexpr (sizeof(word) == 4) *reinterpret_cast<uint32_t *>(st + M::weyl_off + 4) = 0u;
    *reinterpret_cast<uint64_t *>(st + M::pos_off) = pos;
  }
}

// Seeds streams [0, num_streams): stream k from SplitMix64(seed + k) outputs
// 1 .. 64 (ring x_{-64} .. x_{-1}, high w bits) and 65 (the Weyl start); an
// all-zero ring gets x_{-1} = 1; then 4 r = 256 steps are discarded.
template <class M>
__global__ __launch_bounds__(256) void k_fam_init(unsigned char *__restrict__ state, uint64_t num_streams,
                                                  uint64_t seed) {
  using word = typename M::word;
  const Lanes L = lanes_of(num_streams, blockIdx.x);
  if (2 * (L.k >> 1) >= num_streams) return;  // wave-uniform: both streams of the pair absent
  const uint64_t s = seed + L.k;
  word prev = seed_word<M>(splitmix64_at(s, L.j + 1u));
  word cur = seed_word<M>(splitmix64_at(s, L.j + 33u));
  const word w0 = seed_word<M>(splitmix64_at(s, 65u));
  const uint64_t nz = __ballot((prev | cur) != 0);
  const uint64_t mine = L.h ? 0xAAAAAAAAAAAAAAAAull : 0x5555555555555555ull;
  if ((nz & mine) == 0 && L.j == 31u) cur = 1;  // x_{-1} = 1
  Ring2<M> g;
  g.open(prev, cur);
  const bool word0 = L.j == 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) (void)g.step(word0);
  store_state<M>(state + L.k * M::state_bytes, L, g.prev, g.cur, word(0), 0u, w0 + word(256) * M::omega, 0ull);
}

// n words of one stream per half-wavefront from its state at st: the full
// steps go to o, o + stride, ... (o already offset to word j of the step),
// the ragged last step (rem = n mod 32 words) to tail + j, or after the full
// steps when tail is NULL.  on = false masks this lane's loads and stores
// (that half's stream is absent); n is wave-uniform.
template <class M, uint32_t KIND, int UNROLL>
__device__ __forceinline__ void fam_run(unsigned char *__restrict__ st, bool on, Lanes L, uint64_t n,
                                        typename M::word *__restrict__ o, uint64_t stride,
                                        typename M::word *__restrict__ tail) {
  using word = typename M::word;
  L.active = on;
  const word *ring = reinterpret_cast<const word *>(st);
  word prev = 0, cur = 0, w_start = 0;
  uint64_t pos = 0;
  if (on) {
    prev = ring[L.j];
    cur = ring[32 + L.j];
    w_start = *reinterpret_cast<const word *>(st + M::weyl_off);
    pos = *reinterpret_cast<const uint64_t *>(st + M::pos_off);
  }
  Ring2<M> g;
  g.open(prev, cur);
  const bool word0 = L.j == 0;
  const word wlane = word(L.j + 1u) * M::omega;  // W_{p+j} = W_{p-1} + (j + 1) omega
  word wbase = w_start;
  const uint64_t nfull = n / kStep;
  const uint32_t rem = (uint32_t)(n % kStep);
  const uint64_t nouter = nfull / UNROLL;
  for (uint64_t it = 0; it != nouter; ++it) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const word x = g.step(word0);
      const word w = wbase + wlane;
      wbase += word(kStep) * M::omega;
      if (on) __builtin_nontemporal_store(map_out<M, KIND>(x + (word)(w ^ (w >> M::gamma))), o + u * stride);
    }
    o += UNROLL * stride;
  }
  for (uint64_t c = nouter * UNROLL; c != nfull; ++c) {
    const word x = g.step(word0);
    const word w = wbase + wlane;
    wbase += word(kStep) * M::omega;
    if (on) __builtin_nontemporal_store(map_out<M, KIND>(x + (word)(w ^ (w >> M::gamma))), o);
    o += stride;
  }
  const word p0 = g.prev, c0 = g.cur;
  word x = 0;
  if (rem) {  // wave-uniform
    x = g.step(word0);
    const word w = wbase + wlane;
    word *t = tail ? tail : o;
    if (on && L.j < rem) __builtin_nontemporal_store(map_out<M, KIND>(x + (word)(w ^ (w >> M::gamma))), t);
  }
  store_state<M>(st, L, p0, c0, x, rem, w_start + (word)n * M::omega, pos + n);
}

// n words of each of `count` streams (launch index k = stream first + k).
// FILL = false: stream-major, out[k n + t].  FILL = true: chunk c (words
// 32c .. 32c + 31) of stream k at out[(c count + k) 32 ..], the ragged last
// chunks (rem = n mod 32 words each) packed after them at
// out[32 (n / 32) count + k rem ..]; a wavefront's step then writes 64
// adjacent words.  CHECK: the wavefront's second stream is absent (odd count,
// last pair), so that half's loads and stores are masked.
template <class M, uint32_t KIND, int UNROLL, bool FILL, bool CHECK>
__device__ __forceinline__ void fam_serve(unsigned char *__restrict__ state, const Lanes &L, uint64_t first,
                                          uint64_t count, uint64_t n, typename M::word *__restrict__ out) {
  using word = typename M::word;
  const bool on = !CHECK || L.active;
  unsigned char *st = state + (first + L.k) * M::state_bytes;
  if constexpr (FILL) {
    word *tail = out + (n / kStep) * count * kStep + L.k * (n % kStep) + L.j;
    fam_run<M, KIND, UNROLL>(st, on, L, n, out + L.k * kStep + L.j, count * kStep, tail);
  } else {
    fam_run<M, KIND, UNROLL>(st, on, L, n, out + L.k * n + L.j, kStep, nullptr);
  }
}

// ---------------------------------------------------------------------------
// normals: Box-Muller on consecutive pairs (o_{2m}, o_{2m+1}) of each
// stream's outputs of the call, as for Section 2's member; FP32 from the
// 32-bit member, FP64 (53-bit uniforms) from the 64-bit member.  Two steps
// give 64 words of each stream, i.e. 32 pairs: lane 2m + h takes pair m of
// stream h, whose words sit on lanes (4m + h) mod 64 and (4m + 2 + h) mod 64
// of the first step (m < 16) or of the second.  MOMENTS (32-bit member):
// per-lane compensated sums of z and z^2, reduced over the lanes of each
// stream (their lane parity), instead of storing the variates.
// ---------------------------------------------------------------------------
// FP64 normals of the 64-bit member: u1 = ((e >> 11) + 1) 2^-53 in (0, 1]
// and u2 = (o >> 11) 2^-53 in [0, 1), both exact; z0 = rho cos(2 pi u2),
// z1 = rho sin(2 pi u2), rho = sqrt(-2 ln u1).  The angle is reduced exactly
// on the word as in dev::sincos_turn: adding 2^61 to o leaves the quadrant in bits
// 63:62 and (o's low 11 bits cleared) 2^61 + f 2^63 in bits 61:0, |f| <= 1/4.
// sin(pi f), cos(pi f), ln and the square root are the device library's FP64
// functions.
__device__ __forceinline__ void box_muller_f64(uint64_t e, uint64_t o, double &z0, double &z1) {
  const double u1 = fma((double)(e >> 11), 0x1p-53, 0x1p-53);  // exact
  const double rho = sqrt(-2.0 * log(u1));
  const uint64_t qf = o + (1ull << 61);
  const double f = fma((double)(qf & 0x3FFFFFFFFFFFF800ull), 0x1p-63, -0.25);  // exact
  double sp, cp;
  sincospi(f, &sp, &cp);
  const bool odd = ((qf >> 62) & 1u) != 0u;
  const double s0 = odd ? cp : sp, c0 = odd ? sp : cp;
  const uint64_t sign_s = qf & 0x8000000000000000ull, sign_c = (qf + (1ull << 62)) & 0x8000000000000000ull;
  z0 = rho * __longlong_as_double((long long)((uint64_t)__double_as_longlong(c0) ^ sign_c));
  z1 = rho * __longlong_as_double((long long)((uint64_t)__double_as_longlong(s0) ^ sign_s));
}

template <typename word>
__device__ __forceinline__ void fam_gather_pair(word a, word b, uint32_t m, uint32_t h, word &e, word &o) {
  const int se = (int)((4u * m + h) & 63u), so = (int)((4u * m + 2u + h) & 63u);
  const word ea = shfl_word(a, se), eb = shfl_word(b, se), oa = shfl_word(a, so), ob = shfl_word(b, so);
  const bool upper = m >= 16u;
  e = upper ? eb : ea;
  o = upper ? ob : oa;
}

// Compensated FP64 sums of z and z^2 kept by one lane (one update per pair).
struct MomentsF64 {
  double s1, c1, s2, c2;
};

__device__ __forceinline__ void kahan_add_f64(double &s, double &c, double v) {
  const double y = v - c;
  const double t = s + y;
  c = (t - s) - y;
  s = t;
}

// FP64 normals idx and idx + 1 of the call (those below n): stored (a pair is
// one 16-byte store when `pair_aligned`, wave-uniform) or, MOMENTS, added to
// the lane's sums as z0 + z1 and fma(z1, z1, z0 z0).
template <bool MOMENTS>
__device__ __forceinline__ void fam_consume_pair_f64(uint64_t e, uint64_t o, uint64_t idx, uint64_t n, bool on,
                                                     double *__restrict__ out, bool pair_aligned,
                                                     MomentsF64 &m) {
  double z0, z1;
  box_muller_f64(e, o, z0, z1);
  const bool has0 = on && idx < n, has1 = on && idx + 1 < n;
  if constexpr (MOMENTS) {
    if (has0) {  // has1 implies has0
      const double b = has1 ? z1 : 0.0;
      kahan_add_f64(m.s1, m.c1, z0 + b);
      kahan_add_f64(m.s2, m.c2, fma(b, b, z0 * z0));
    }
  } else if (pair_aligned && has1) {
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    const f64x2 pair = {z0, z1};
    __builtin_nontemporal_store(pair, reinterpret_cast<f64x2 *>(out + idx));
  } else {
    if (has0) __builtin_nontemporal_store(z0, out + idx);
    if (has1) __builtin_nontemporal_store(z1, out + idx + 1);
  }
}

template <bool MOMENTS>
__device__ __forceinline__ void fam_consume_pair(uint32_t e, uint32_t o, uint64_t idx, uint64_t n, bool on,
                                                 float *__restrict__ out, bool pair_aligned, dev::Moments &m) {
  float z0, z1;
  dev::box_muller(e, o, z0, z1);
  const bool has0 = on && idx < n, has1 = on && idx + 1 < n;
  if constexpr (MOMENTS) {
    if (has0) {  // a group of one pair per compensated update (has1 implies has0)
      dev::group_add(m, z0, has1 ? z1 : 0.0f);
      dev::group_close(m);
    }
  } else {
    if (pair_aligned && has1) {
      typedef float f32x2 __attribute__((ext_vector_type(2)));
      const f32x2 pair = {z0, z1};
      __builtin_nontemporal_store(pair, reinterpret_cast<f32x2 *>(out + idx));
    } else {
      if (has0) __builtin_nontemporal_store(z0, out + idx);
      if (has1) __builtin_nontemporal_store(z1, out + idx + 1);
    }
  }
}

// n normals of each of `count` streams (launch index k = stream first + k)
// at out[k n + t], or their sums at sums[2k], sums[2k + 1].  Consumes
// 2 ceil(n / 2) words per stream.
// n normals of the stream at st per half-wavefront (n wave-uniform), from
// 2 ceil(n / 2) words: Box-Muller on consecutive pairs, written from o_s
// (the stream's first output) unless MOMENTS, which instead reduces the
// half's sums of z and z^2 and stores them at sums (two reals).  on = false
// masks this lane's loads and stores.
template <class M, bool MOMENTS>
__device__ __forceinline__ void fam_normals_run(unsigned char *__restrict__ st, bool on, Lanes L, uint64_t n,
                                                typename std::conditional<sizeof(typename M::word) == 8, double,
                                                                          float>::type *__restrict__ o_s,
                                                typename std::conditional<sizeof(typename M::word) == 8, double,
                                                                          float>::type *__restrict__ sums) {
  using word = typename M::word;
  constexpr bool kW64 = sizeof(word) == 8;
  using real = typename std::conditional<kW64, double, float>::type;
  L.active = on;
  word prev = 0, cur = 0, w_start = 0;
  uint64_t pos = 0;
  if (on) {
    const word *ring = reinterpret_cast<const word *>(st);
    prev = ring[L.j];
    cur = ring[32 + L.j];
    w_start = *reinterpret_cast<const word *>(st + M::weyl_off);
    pos = *reinterpret_cast<const uint64_t *>(st + M::pos_off);
  }
  Ring2<M> g;
  g.open(prev, cur);
  const bool word0 = L.j == 0;
  const word wlane = word(L.j + 1u) * M::omega;
  word wbase = w_start;
  auto next = [&]() {
    const word x = g.step(word0);
    const word w = wbase + wlane;
    wbase += word(kStep) * M::omega;
    return word(x + (w ^ (w >> M::gamma)));
  };
  const uint64_t words = n + (n & 1u);
  const uint64_t nblk = words >> 6;  // 64-word blocks: 32 pairs of each stream
  const uint32_t rw = (uint32_t)(words & 63u);
  const uint32_t m = L.j;
  const bool pair_aligned =
      !MOMENTS && (n & 1u) == 0 && (reinterpret_cast<uintptr_t>(o_s) & (2 * sizeof(real) - 1)) == 0;
  dev::Moments mo{0.0f, 0.0f, 0.0f, 0.0f, -0.0f, -0.0f};
  MomentsF64 md{0.0, 0.0, 0.0, 0.0};
  auto consume = [&](word e, word o, uint64_t idx) {
    if constexpr (kW64) fam_consume_pair_f64<MOMENTS>(e, o, idx, n, on, o_s, pair_aligned, md);
    else fam_consume_pair<MOMENTS>(e, o, idx, n, on, o_s, pair_aligned, mo);
  };
  uint64_t b = 0;
  if constexpr (MOMENTS && !kW64) {
    // Blocks wholly below n, four at a time: each pair enters the sums
    // unordered and unchecked (a masked half's sums are never stored), and
    // each group of four pairs takes one compensated update.
    for (const uint64_t nsafe4 = (n >> 6) & ~uint64_t(3); b != nsafe4; b += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const word oa = next();
        const word ob = next();
        word e, o;
        fam_gather_pair(oa, ob, m, L.h, e, o);
        float za, zb;
        dev::box_muller_unordered(e, o, za, zb);
        dev::group_add(mo, za, zb);
      }
      dev::group_close(mo);
    }
  }
  for (; b != nblk; ++b) {
    const word oa = next();
    const word ob = next();
    word e, o;
    fam_gather_pair(oa, ob, m, L.h, e, o);
    consume(e, o, (b << 6) + 2u * m);
  }
  // Tail: rw (even, < 64) more words.
  word p0 = g.prev, c0 = g.cur, xl = 0;
  uint32_t rem = 0u;
  if (rw) {  // wave-uniform
    word oa, ob = 0;
    if (rw <= 32u) {
      const word w = wbase + wlane;
      xl = g.step(word0);
      oa = xl + (w ^ (w >> M::gamma));
      rem = rw & 31u;  // rw == 32 completes the step
      if (!rem) {
        p0 = g.prev;
        c0 = g.cur;
      }
    } else {
      oa = next();
      p0 = g.prev;
      c0 = g.cur;
      const word w = wbase + wlane;
      xl = g.step(word0);
      ob = xl + (w ^ (w >> M::gamma));
      rem = rw - 32u;
    }
    word e, o;
    fam_gather_pair(oa, ob, m, L.h, e, o);
    if (2u * m < rw) consume(e, o, (nblk << 6) + 2u * m);
  }
  store_state<M>(st, L, p0, c0, xl, rem, w_start + (word)words * M::omega, pos + words);
  if constexpr (MOMENTS) {
    // Folded and reduced across the stream's lanes in FP64 (for the FP32
    // sums: rounded once to FP32 at the end).
    double v1, v2;
    if constexpr (kW64) {
      v1 = md.s1 - md.c1;
      v2 = md.s2 - md.c2;
    } else {
      v1 = (double)mo.s1 - (double)mo.c1;
      v2 = (double)mo.s2 - (double)mo.c2;
    }
#pragma unroll
    for (int off = 32; off >= 2; off >>= 1) {  // even offsets keep each stream's lanes apart
      v1 += __shfl_xor(v1, off);
      v2 += __shfl_xor(v2, off);
    }
    if (on && L.j == 0) {
      sums[0] = (real)v1;
      sums[1] = (real)v2;
    }
  }
}

template <class M, bool MOMENTS>
__global__ __launch_bounds__(1024) void k_fam_normals(unsigned char *__restrict__ state, uint64_t first,
                                                      uint64_t count, uint64_t n, void *__restrict__ out_v,
                                                      void *__restrict__ sums_v) {
  using word = typename M::word;
  using real = typename std::conditional<sizeof(word) == 8, double, float>::type;
  real *out = static_cast<real *>(out_v);
  real *sums = static_cast<real *>(sums_v);
  const Lanes L = lanes_of(count, xcd_block());
  if (2 * (L.k >> 1) >= count) return;  // wave-uniform
  fam_normals_run<M, MOMENTS>(state + (first + L.k) * M::state_bytes, L.active, L, n,
                              MOMENTS ? nullptr : out + L.k * n, MOMENTS ? sums + 2 * L.k : nullptr);
}

template <class M, uint32_t KIND, int UNROLL, bool FILL>
__global__ __launch_bounds__(1024) void k_fam_generate(unsigned char *__restrict__ state, uint64_t first,
                                                       uint64_t count, uint64_t n, void *__restrict__ out) {
  // Stream-major: each XCD takes a contiguous range of streams; bulk fill:
  // plain order, so every XCD's writes spread over the whole dense front
  // (each measured the faster for its layout).
  const Lanes L = lanes_of(count, FILL ? blockIdx.x : xcd_block());
  const uint64_t pair = L.k >> 1;
  if (2 * pair >= count) return;  // wave-uniform
  using word = typename M::word;
  if (2 * pair + 1 < count)
    fam_serve<M, KIND, UNROLL, FILL, false>(state, L, first, count, n, reinterpret_cast<word *>(out));
  else
    fam_serve<M, KIND, UNROLL, FILL, true>(state, L, first, count, n, reinterpret_cast<word *>(out));
}

// ---------------------------------------------------------------------------
// Batched requests (the persistent launch of xg_generate_batch) for these
// members.  A wavefront serves two request groups at once, one per
// half-wavefront (lanes 2j + h serve group 2p + h of pair p: first the pair
// of the wavefront's own index in the grid, then pairs taken from the atomic
// queue work[0]).  Each loop trip runs min(words left in the two
// current requests) through fam_run, with the state written back between
// trips, so both halves step together; a half whose group is done, or whose
// current request has the other output type, is masked for that trip (half
// 0 goes first).  While a half's next word falls inside a 32-word line of the
// output, a one-step head trip (fam_head) first brings each such half to its
// line's end, so that full steps store whole aligned lines.  Requests are
// uint32 / uint64 (XG_U32), FP32 / FP64 (XG_F32) or normals of that precision
// (XG_NORMAL), in elements of the member's word width; a request or group
// that fails the bounds check (stream, dtype, flags 0, output range, group
// offsets) is skipped and sets work[1].  Every wavefront exits once the queue
// passes work[2] groups.
// ---------------------------------------------------------------------------
// One generator step of the stream at st, of which this half writes the
// first `head` words (head < 32, per half; 0 writes nothing and leaves the
// state as it was) as integers or, if real, as uniform reals; the state then
// stands `head` words further on.  Branch-free in head, so every lane takes
// part in the shuffles.
template <class M, uint32_t KINT, uint32_t KREAL>
__device__ __forceinline__ void fam_head(unsigned char *__restrict__ st, bool on, const Lanes &L, uint32_t head,
                                         bool real, typename M::word *__restrict__ o) {
  using word = typename M::word;
  word *ring = reinterpret_cast<word *>(st);
  word prev = 0, cur = 0, w_start = 0;
  uint64_t pos = 0;
  if (on) {
    prev = ring[L.j];
    cur = ring[32 + L.j];
    w_start = *reinterpret_cast<const word *>(st + M::weyl_off);
    pos = *reinterpret_cast<const uint64_t *>(st + M::pos_off);
  }
  Ring2<M> g;
  g.open(prev, cur);
  const word x = g.step(L.j == 0);
  const word w = w_start + word(L.j + 1u) * M::omega;
  const word v = x + (word)(w ^ (w >> M::gamma));
  if (on && L.j < head) __builtin_nontemporal_store(real ? map_out<M, KREAL>(v) : map_out<M, KINT>(v), o);
  // The new ring: the 64-word window ending `head` words into x.
  const uint32_t js = (head + L.j) & 31u;
  const int src = (int)(2 * js + L.h);
  const word a = shfl_word(prev, src), b = shfl_word(cur, src), c = shfl_word(x, src);
  const bool wrap = head + L.j >= 32u;
  if (!on) return;
  ring[L.j] = wrap ? b : a;
  ring[32 + L.j] = wrap ? c : b;
  if (L.j == 0) {
    *reinterpret_cast<word *>(st + M::weyl_off) = w_start + (word)head * M::omega;
    *reinterpret_cast<uint64_t *>(st + M::pos_off) = pos + head;
  }
}

// Lane src's value of v, held in scalar registers.
__device__ __forceinline__ uint64_t lane_value(uint64_t v, int src) {
  const uint64_t x = shfl_word(v, src);
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32)) << 32) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
}

template <class M, int UNROLL>
__global__ __launch_bounds__(1024) void k_fam_batch(unsigned char *__restrict__ state, uint64_t num_streams,
                                                    const xg_request *__restrict__ reqs,
                                                    const uint32_t *__restrict__ groups,
                                                    void *__restrict__ out_v, uint64_t out_elems,
                                                    uint32_t *__restrict__ work) {
  const uint32_t num_groups = work[2], num_reqs = work[3];
  using word = typename M::word;
  constexpr uint32_t kInt = sizeof(word) == 4 ? kU32 : kU64;
  constexpr uint32_t kReal = sizeof(word) == 4 ? kF32 : kF64;
  using real = typename std::conditional<sizeof(word) == 8, double, float>::type;
  word *out = reinterpret_cast<word *>(out_v);
  Lanes L;
  L.lane = threadIdx.x & 63u;
  L.h = L.lane & 1u;
  L.j = L.lane >> 1;
  L.k = 0;
  L.active = true;
  // Queue items are pairs of groups (one per half), largest first; a
  // wavefront takes `take` consecutive pairs per atomic, as k_batch does.
  // The first pair is the wavefront's own index in the grid; later trips
  // take pairs from the counter, offset by the wavefronts in the grid.
  const uint32_t num_pairs = (uint32_t)((num_groups + 1ull) / 2);
  const uint32_t wpb = blockDim.x >> 6;
  const uint32_t waves = gridDim.x * wpb;
  uint32_t p0 = blockIdx.x * wpb + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint32_t take = 1;
  for (;;) {
    if (p0 >= num_pairs) break;
    const uint32_t p_end = num_pairs - p0 < take ? num_pairs : p0 + take;
    uint64_t served = 0;  // words of the trips run for these pairs
    for (uint32_t p = p0; p < p_end; ++p) {
      const uint64_t g = 2ull * p + L.h;
      uint32_t r = 0, r_end = 0;
      if (g < num_groups) {
        r = groups[g];
        r_end = groups[g + 1];
        if (r > r_end || r_end > num_reqs) {
          if (L.j == 0) atomicOr(&work[1], 1u);
          r = r_end = 0;
        }
      }
      uint64_t done = 0;  // words of the half's current request already written
      for (;;) {
        // Each half moves past bad and empty requests (no cross-lane work here).
        xg_request q{};
        bool have = false;
        while (r < r_end) {
          q = reqs[r];
          const bool ok = q.stream < num_streams && q.dtype <= XG_NORMAL && q.flags == 0u &&
                          q.out_offset <= out_elems && q.n <= out_elems - q.out_offset;
          if (ok && q.n > done) {
            have = true;
            break;
          }
          if (!ok && L.j == 0) atomicOr(&work[1], 1u);
          ++r;
          done = 0;
        }
        const uint64_t left = have ? q.n - done : 0;
        const uint64_t left0 = lane_value(left, 0), left1 = lane_value(left, 1);
        if (left0 == 0 && left1 == 0) break;
        // Position of the half's next word within a 32-word line of the output.
        // (Normals are written pair by pair and are not realigned.)
        const uint32_t mis = have && q.dtype != XG_NORMAL
                                 ? (uint32_t)((reinterpret_cast<uintptr_t>(out) / sizeof(word) + q.out_offset + done) % kStep)
                                 : 0u;
        const uint32_t mis0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl((int)mis, 0));
        const uint32_t mis1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl((int)mis, 1));
        if (mis0 != 0u || mis1 != 0u) {
          // Head trip: one step, in which each half that starts inside a line
          // writes only up to that line's end, so its later full steps store
          // whole aligned lines (dense request offsets start most requests
          // inside a line, which measured twice as slow).
          const uint32_t head = mis != 0u ? (uint32_t)(left < kStep - mis ? left : kStep - mis) : 0u;
          const bool mine = head != 0u;
          unsigned char *st = state + (mine ? q.stream : 0) * M::state_bytes;
          word *o = out + (mine ? q.out_offset + done : 0) + L.j;
          fam_head<M, kInt, kReal>(st, mine, L, head, q.dtype == XG_F32, o);
          if (mine) {
            done += head;
            if (done == q.n) {
              ++r;
              done = 0;
            }
          }
          continue;
        }
        const uint32_t dt0 = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)q.dtype, 0));
        const uint32_t dt1 = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)q.dtype, 1));
        bool run0 = left0 != 0;
        bool run1 = left1 != 0 && (!run0 || dt0 == dt1);
        uint64_t n = run0 ? (run1 && left1 < left0 ? left1 : left0) : left1;
        const uint32_t kind = run0 ? dt0 : dt1;
        if (kind == XG_NORMAL && (n & 1u)) {
          // An odd count drops the second variate of its last pair, so only a
          // half that finishes its request with this trip may take one.
          const bool fin0 = run0 && left0 == n, fin1 = run1 && left1 == n;
          if ((run0 && !fin0) || (run1 && !fin1)) {
            if (n > 1) {
              n -= 1;
            } else {
              run0 = fin0;
              run1 = fin1;
            }
          }
        }
        const bool mine = L.h ? run1 : run0;
        unsigned char *st = state + (mine ? q.stream : 0) * M::state_bytes;
        const uint64_t at = mine ? q.out_offset + done : 0;
        if (kind == XG_NORMAL)
          fam_normals_run<M, false>(st, mine, L, n, reinterpret_cast<real *>(out) + at, nullptr);
        else if (kind == XG_F32)
          fam_run<M, kReal, UNROLL>(st, mine, L, n, out + at + L.j, kStep, nullptr);
        else
          fam_run<M, kInt, UNROLL>(st, mine, L, n, out + at + L.j, kStep, nullptr);
        served += n;
        if (mine) {
          done += n;
          if (done == q.n) {
            ++r;
            done = 0;
          }
        }
      }
    }
    const uint64_t budget = kBatchTakeWords * (p_end - p0);
    take = 1;
    while (take < kBatchMaxTake && served * (2u * take) <= budget) take <<= 1;
    uint32_t c = 0;
    if (L.lane == 0) c = atomicAdd(&work[0], take);
    p0 = waves + (uint32_t)__builtin_amdgcn_readfirstlane((int)c);
  }
}

template <class M>
hipError_t launch_fam_batch_k(uint32_t unroll, uint64_t blocks, dim3 block, int num_cus, unsigned char *state,
                              uint64_t num_streams, const xg_request *reqs, const uint32_t *groups, void *out,
                              uint64_t out_elems, uint32_t *work, hipStream_t stream) {
  auto run = [&](auto kernel) {
    return launch_persistent(kernel, blocks, block, 0, num_cus, stream, state, num_streams, reqs, groups, out,
                             out_elems, work);
  };
  switch (unroll) {
    case 1: return run(k_fam_batch<M, 1>);
    case 2: return run(k_fam_batch<M, 2>);
    case 4: return run(k_fam_batch<M, 4>);
    default: return run(k_fam_batch<M, 8>);
  }
}

// ---------------------------------------------------------------------------
// skip: advance each stream by J words without producing them.
//
// JUMP = false: the x-part steps through the J words (J small).
// JUMP = true: T^J = g(T), g = z^J mod P of degree < n (Cayley-Hamilton), is
// evaluated on the state S0 by Horner's rule in steps of 32 words:
//   S <- T^32 S  xor  sum_{i < 32} g_{32c + i} T^i S0,   c = n/32 - 1 .. 0.
// T^32 S is one generator step of the x-part.  T^i S0 is the 64-word window
// starting i words into S0's continuation E = ring | the next 32 words, so
// lane 2j + h needs E[j .. j + 63] of its stream: E is staged through LDS once
// and kept in registers.  The bits of g are wave-uniform (both streams of a
// wavefront jump by the same J).  W advances by J omega and pos by J.
// ---------------------------------------------------------------------------
extern __shared__ __align__(16) unsigned char fam_lds[];

template <class M, bool JUMP>
__global__ __launch_bounds__(256) void k_fam_skip(unsigned char *__restrict__ state, uint64_t first,
                                                  uint64_t count, uint64_t J, JumpPoly g) {
  using word = typename M::word;
  constexpr uint32_t kN = 64u * 8u * sizeof(word);  // n = r w with r = 64
  const Lanes L = lanes_of(count, blockIdx.x);
  if (2 * (L.k >> 1) >= count) return;  // wave-uniform
  unsigned char *st = state + (first + L.k) * M::state_bytes;
  word prev = 0, cur = 0, w_start = 0;
  uint64_t pos = 0;
  if (L.active) {
    const word *ring = reinterpret_cast<const word *>(st);
    prev = ring[L.j];
    cur = ring[32 + L.j];
    w_start = *reinterpret_cast<const word *>(st + M::weyl_off);
    pos = *reinterpret_cast<const uint64_t *>(st + M::pos_off);
  }
  const bool word0 = L.j == 0;
  const word w_end = w_start + (word)J * M::omega;
  if constexpr (!JUMP) {
    Ring2<M> r;
    r.open(prev, cur);
    const uint64_t nfull = J / kStep;
    const uint32_t rem = (uint32_t)(J % kStep);
    for (uint64_t c = 0; c != nfull; ++c) (void)r.step(word0);
    const word p0 = r.prev, c0 = r.cur;
    word x = 0;
    if (rem) x = r.step(word0);
    store_state<M>(st, L, p0, c0, x, rem, w_end, pos + J);
  } else {
    Ring2<M> r;
    r.open(prev, cur);
    const word nxt = r.step(word0);            // x_{p+j}: the continuation's next 32 words
    word *E = reinterpret_cast<word *>(fam_lds) + (threadIdx.x >> 6) * 192u + L.h * 96u;
    E[L.j] = prev;
    E[32 + L.j] = cur;
    E[64 + L.j] = nxt;
    dev::wave_lds_sync();                      // the reads below take other lanes' words
    word e[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) e[i] = E[L.j + i];
    word sp = 0, sc = 0;                       // S: words j and 32 + j of the accumulated state
    for (int c = (int)(kN / kStep) - 1; c >= 0; --c) {
      if (c != (int)(kN / kStep) - 1) {
        Ring2<M> t;
        t.open(sp, sc);
        const word x = t.step(word0);
        sp = sc;
        sc = x;
      }
      const uint32_t bits = (uint32_t)(g.w[c >> 1] >> ((c & 1) * 32));
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        const word m = (word)0 - (word)((bits >> i) & 1u);
        sp ^= e[i] & m;
        sc ^= e[32 + i] & m;
      }
    }
    store_state<M>(st, L, sp, sc, word(0), 0u, w_end, pos + J);
  }
}

template <class M, uint32_t KIND, bool FILL>
hipError_t launch_fam_k(uint32_t unroll, dim3 grid, dim3 block, unsigned char *state, uint64_t first,
                  uint64_t count, uint64_t n, void *out, hipStream_t stream) {
  hipError_t e = hipSuccess;
  switch (unroll) {
    case 1: e = launch((k_fam_generate<M, KIND, 1, FILL>), grid, block, 0, stream, state, first, count, n, out); break;
    case 2: e = launch((k_fam_generate<M, KIND, 2, FILL>), grid, block, 0, stream, state, first, count, n, out); break;
    case 4: e = launch((k_fam_generate<M, KIND, 4, FILL>), grid, block, 0, stream, state, first, count, n, out); break;
    default: e = launch((k_fam_generate<M, KIND, 8, FILL>), grid, block, 0, stream, state, first, count, n, out); break;
  }
  return e;
}

template <class M, uint32_t KIND>
hipError_t launch_fam_layout(bool fill, uint32_t unroll, dim3 grid, dim3 block, unsigned char *state,
                             uint64_t first, uint64_t count, uint64_t n, void *out, hipStream_t stream) {
  if (fill) return launch_fam_k<M, KIND, true>(unroll, grid, block, state, first, count, n, out, stream);
  return launch_fam_k<M, KIND, false>(unroll, grid, block, state, first, count, n, out, stream);
}

}  // namespace

uint32_t family_state_bytes(uint32_t family) {
  switch (family) {
    case XG_FAMILY_R128_W32: return XG_STATE_WORDS * 4;
    case XG_FAMILY_R64_W32: return MemberN2048::state_bytes;
    case XG_FAMILY_R64_W64: return MemberW64::state_bytes;
    default: return 0;
  }
}

uint32_t family_pos_offset(uint32_t family) {
  switch (family) {
    case XG_FAMILY_R128_W32: return 130 * 4;
    case XG_FAMILY_R64_W32: return MemberN2048::pos_off;
    case XG_FAMILY_R64_W64: return MemberW64::pos_off;
    default: return 0;
  }
}

hipError_t launch_family_init(uint32_t family, unsigned char *state, uint64_t num_streams, uint64_t seed,
                              hipStream_t stream) {
  hipError_t e = hipSuccess;
  const uint64_t pairs = (num_streams + 1) / 2;
  const dim3 grid((uint32_t)((pairs + 3) / 4)), block(256);
  if (family == XG_FAMILY_R64_W32)
    e = launch(k_fam_init<MemberN2048>, grid, block, 0, stream, state, num_streams, seed);
  else if (family == XG_FAMILY_R64_W64)
    e = launch(k_fam_init<MemberW64>, grid, block, 0, stream, state, num_streams, seed);
  else
    return hipErrorInvalidValue;
  return e;
}

hipError_t launch_family_skip(uint32_t family, unsigned char *state, uint64_t first, uint64_t count, uint64_t J,
                              const JumpPoly *g, hipStream_t stream) {
  hipError_t e = hipSuccess;
  const uint64_t pairs = (count + 1) / 2;
  const dim3 grid((uint32_t)((pairs + 3) / 4)), block(256);
  JumpPoly zero{};
  const JumpPoly &gp = g ? *g : zero;
  if (family == XG_FAMILY_R64_W32) {
    if (g) e = launch((k_fam_skip<MemberN2048, true>), grid, block, 4 * 192 * 4, stream, state, first, count, J, gp);
    else e = launch((k_fam_skip<MemberN2048, false>), grid, block, 0, stream, state, first, count, J, gp);
  } else if (family == XG_FAMILY_R64_W64) {
    if (g) e = launch((k_fam_skip<MemberW64, true>), grid, block, 4 * 192 * 8, stream, state, first, count, J, gp);
    else e = launch((k_fam_skip<MemberW64, false>), grid, block, 0, stream, state, first, count, J, gp);
  } else {
    return hipErrorInvalidValue;
  }
  return e;
}

hipError_t launch_family_generate(uint32_t family, Kind kind, bool fill, const Shape &shape, unsigned char *state,
                                  uint64_t first, uint64_t count, uint64_t n, void *out, hipStream_t stream) {
  hipError_t e = hipSuccess;
  const uint64_t pairs = (count + 1) / 2;
  const uint64_t wpb = shape.waves_per_block;
  const dim3 grid((uint32_t)((pairs + wpb - 1) / wpb)), block((uint32_t)(wpb * kWave));
  if (family == XG_FAMILY_R64_W32 && (kind == kNormal || kind == kMoments)) {
    float *o = static_cast<float *>(out);
    if (kind == kNormal)
      e = launch((k_fam_normals<MemberN2048, false>), grid, block, 0, stream, state, first, count, n, out,
                         nullptr);
    else
      e = launch((k_fam_normals<MemberN2048, true>), grid, block, 0, stream, state, first, count, n, nullptr,
                         o);
    return e;
  }
  if (family == XG_FAMILY_R64_W64 && (kind == kNormal || kind == kMoments)) {
    if (kind == kNormal)
      e = launch((k_fam_normals<MemberW64, false>), grid, block, 0, stream, state, first, count, n, out,
                         nullptr);
    else
      e = launch((k_fam_normals<MemberW64, true>), grid, block, 0, stream, state, first, count, n, nullptr,
                         out);
    return e;
  }
  if (family == XG_FAMILY_R64_W32 && kind == kU32)
    e = launch_fam_layout<MemberN2048, kU32>(fill, shape.unroll, grid, block, state, first, count, n, out, stream);
  else if (family == XG_FAMILY_R64_W32 && kind == kF32)
    e = launch_fam_layout<MemberN2048, kF32>(fill, shape.unroll, grid, block, state, first, count, n, out, stream);
  else if (family == XG_FAMILY_R64_W64 && kind == kU64)
    e = launch_fam_layout<MemberW64, kU64>(fill, shape.unroll, grid, block, state, first, count, n, out, stream);
  else if (family == XG_FAMILY_R64_W64 && kind == kF64)
    e = launch_fam_layout<MemberW64, kF64>(fill, shape.unroll, grid, block, state, first, count, n, out, stream);
  else
    return hipErrorInvalidValue;
  return e;
}

hipError_t launch_family_batch(uint32_t family, const Shape &shape, int num_cus, unsigned char *state,
                               uint64_t num_streams, const xg_request *reqs, const uint32_t *groups,
                               uint32_t max_groups, void *out, uint64_t out_elems, uint32_t *work,
                               hipStream_t stream) {
  if (family != XG_FAMILY_R64_W32 && family != XG_FAMILY_R64_W64) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  const uint64_t pairs = ((uint64_t)max_groups + 1) / 2;
  uint64_t blocks = (uint64_t)(num_cus > 0 ? num_cus : 1) * shape.blocks_per_cu;
  const uint64_t need = (pairs + shape.waves_per_block - 1) / shape.waves_per_block;
  if (need < blocks) blocks = need ? need : 1;
  const dim3 block(shape.waves_per_block * kWave);
  if (family == XG_FAMILY_R64_W32)
    e = launch_fam_batch_k<MemberN2048>(shape.unroll, blocks, block, num_cus, state, num_streams, reqs, groups, out,
                                        out_elems, work, stream);
  else
    e = launch_fam_batch_k<MemberW64>(shape.unroll, blocks, block, num_cus, state, num_streams, reqs, groups, out,
                                      out_elems, work, stream);
  return e;
}

}  // namespace xg
