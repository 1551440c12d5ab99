// Host side of jump-ahead (libxg): the characteristic polynomial P of the
// x-part's step and the jump polynomials z^J mod P.
//
// The x-part of xorgens is GF(2)-linear (Section 1.5 / Section 2 of
// arXiv:1108.0486): its 4096-bit state moves by a fixed matrix T, and by
// Cayley-Hamilton T^J = g(T) with g = z^J mod P, deg g < 4096.  The device
// evaluates g(T) applied to a stream's state (k_skip).  P is obtained once per
// process from the library's own host stepping of the recurrence, by
// Berlekamp-Massey on one output bit (the minimal polynomial of that bit
// sequence is P because P is irreducible of degree 4096).
#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "xg_host.h"

namespace xg {
namespace {

constexpr int kDeg = 4096;          // r w
constexpr int kW = kDeg / 64;       // words of a residue (degree < 4096)
constexpr int kPW = kW + 1;         // words of P (degree 4096)

// Carry-less 64 x 64 -> 128 product: with the CPU instruction when present.
__attribute__((target("pclmul,sse4.1"))) void clmul_hw(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi) {
  typedef long long v2di __attribute__((vector_size(16)));
  v2di x = {(long long)a, 0}, y = {(long long)b, 0};
  v2di r = __builtin_ia32_pclmulqdq128(x, y, 0x00);
  lo = (uint64_t)r[0];
  hi = (uint64_t)r[1];
}

void clmul_sw(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi) {
  uint64_t l = 0, h = 0;
  for (int i = 0; i < 64; ++i)
    if ((a >> i) & 1u) {
      l ^= b << i;
      if (i) h ^= b >> (64 - i);
    }
  lo = l;
  hi = h;
}

bool have_pclmul() {
  static const bool yes = __builtin_cpu_supports("pclmul") && __builtin_cpu_supports("sse4.1");
  return yes;
}

// out[0 .. wa + wb) = a * b over GF(2).
void pmul(const uint64_t *a, int wa, const uint64_t *b, int wb, uint64_t *out) {
  std::memset(out, 0, sizeof(uint64_t) * (size_t)(wa + wb));
  const bool hw = have_pclmul();
  for (int i = 0; i < wa; ++i) {
    if (!a[i]) continue;
    for (int j = 0; j < wb; ++j) {
      uint64_t lo, hi;
      if (hw) clmul_hw(a[i], b[j], lo, hi); else clmul_sw(a[i], b[j], lo, hi);
      out[i + j] ^= lo;
      out[i + j + 1] ^= hi;
    }
  }
}

// Host stepping of the x-part (Section 2) from a fixed non-zero ring; writes
// bit 0 of x_0 .. x_{nbits-1}.
void xpart_bit0(std::vector<uint8_t> &bits) {
  uint32_t ring[128];
  for (uint32_t i = 0; i < 128; ++i) ring[i] = 0x9E3779B9u * (i + 1) ^ (i << 7);
  uint32_t head = 0;  // slot of x_{k-128}
  for (size_t k = 0; k < bits.size(); ++k) {
    const uint32_t xr = ring[head], xs = ring[(head + 63) & 127];  // x_{k-128}, x_{k-65}
    uint32_t t = xr ^ (xr << 15);
    t ^= t >> 14;
    uint32_t v = xs ^ (xs << 12);
    v ^= v >> 17;
    const uint32_t x = t ^ v;
    ring[head] = x;
    head = (head + 1) & 127;
    bits[k] = (uint8_t)(x & 1u);
  }
}

// Minimal polynomial (as z^L + c_1 z^{L-1} + ... + c_L) of a bit sequence.
int min_poly(const std::vector<uint8_t> &s, std::vector<uint64_t> &poly) {
  const int N = (int)s.size();
  std::vector<uint8_t> C(N + 2, 0), B(N + 2, 0), T;
  C[0] = B[0] = 1;
  int L = 0, m = 1;
  for (int k = 0; k < N; ++k) {
    int d = s[k];
    for (int i = 1; i <= L; ++i) d ^= C[i] & s[k - i];
    if (!d) {
      ++m;
      continue;
    }
    if (2 * L <= k) {
      T = C;
      for (int i = 0; i + m <= N + 1; ++i) C[i + m] ^= B[i];
      L = k + 1 - L;
      B = T;
      m = 1;
    } else {
      for (int i = 0; i + m <= N + 1; ++i) C[i + m] ^= B[i];
      ++m;
    }
  }
  poly.assign((size_t)L / 64 + 1, 0);
  for (int i = 0; i <= L; ++i)
    if (C[i]) poly[(size_t)(L - i) / 64] |= 1ull << ((L - i) % 64);
  return L;
}

struct Modulus {
  uint64_t P[kPW];
  uint64_t mu[kPW];  // floor(z^8192 / P)
  bool ok = false;
};

Modulus g_mod;
std::once_flag g_once;

void init_modulus() {
  std::vector<uint8_t> bits(2 * kDeg + 128);
  xpart_bit0(bits);
  std::vector<uint64_t> poly;
  if (min_poly(bits, poly) != kDeg || poly.size() != (size_t)kPW) return;
  std::memcpy(g_mod.P, poly.data(), sizeof(g_mod.P));
  // mu by long division of z^(2 deg) by P
  std::vector<uint64_t> rem(2 * kPW + 1, 0);
  rem[(2 * kDeg) / 64] |= 1ull << ((2 * kDeg) % 64);
  std::memset(g_mod.mu, 0, sizeof(g_mod.mu));
  for (int i = 2 * kDeg; i >= kDeg; --i) {
    if (!((rem[i / 64] >> (i % 64)) & 1u)) continue;
    g_mod.mu[(i - kDeg) / 64] |= 1ull << ((i - kDeg) % 64);
    const int sh = i - kDeg;
    for (int j = 0; j <= kDeg; ++j)
      if ((g_mod.P[j / 64] >> (j % 64)) & 1u) rem[(j + sh) / 64] ^= 1ull << ((j + sh) % 64);
  }
  g_mod.ok = true;
}

// out = a >> sh for a of wa words, ow output words.
void shr(const uint64_t *a, int wa, int sh, uint64_t *out, int ow) {
  const int q = sh / 64, r = sh % 64;
  for (int i = 0; i < ow; ++i) {
    const uint64_t lo = i + q < wa ? a[i + q] : 0, hi = i + q + 1 < wa ? a[i + q + 1] : 0;
    out[i] = r ? (lo >> r) | (hi << (64 - r)) : lo;
  }
}

// out = a * b mod P (exact Barrett reduction: q = floor(floor(ab / z^n) mu / z^n)).
void mulmod(const uint64_t *a, const uint64_t *b, uint64_t *out) {
  uint64_t prod[2 * kW], h[kPW], t[2 * kPW], q[kPW], qp[2 * kPW];
  pmul(a, kW, b, kW, prod);
  shr(prod, 2 * kW, kDeg, h, kPW);
  pmul(h, kPW, g_mod.mu, kPW, t);
  shr(t, 2 * kPW, kDeg, q, kPW);
  pmul(q, kPW, g_mod.P, kPW, qp);
  for (int i = 0; i < kW; ++i) out[i] = prod[i] ^ qp[i];
}

}  // namespace

bool jump_polynomial(uint64_t J, uint64_t g[64]) {
  std::call_once(g_once, init_modulus);
  if (!g_mod.ok) return false;
  uint64_t base[kW] = {0}, acc[kW] = {0}, tmp[kW];
  base[0] = 2;  // z
  acc[0] = 1;
  while (J) {
    if (J & 1u) {
      mulmod(acc, base, tmp);
      std::memcpy(acc, tmp, sizeof(acc));
    }
    J >>= 1;
    if (J) {
      mulmod(base, base, tmp);
      std::memcpy(base, tmp, sizeof(base));
    }
  }
  std::memcpy(g, acc, sizeof(acc));
  return true;
}

}  // namespace xg
