// Host side of jump-ahead (libxg): the characteristic polynomial P of each
// family member's x-part step and the jump polynomials z^J mod P.
//
// The x-part of xorgens is GF(2)-linear (Section 1.5 / Section 2 of
// arXiv:1108.0486): its n-bit state (n = r w) moves by a fixed matrix T, and
// by Cayley-Hamilton T^J = g(T) with g = z^J mod P, deg g < n.  The device
// evaluates g(T) applied to a stream's state.  P is obtained once per process
// and member from the library's own host stepping of the recurrence, by
// Berlekamp-Massey on one output bit (the minimal polynomial of that bit
// sequence is P because P is irreducible of degree n).
#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "xg_host.h"

namespace xg {
namespace {

constexpr int kMaxDeg = 4096;
constexpr int kMaxW = kMaxDeg / 64;  // words of a residue (degree < 4096)
constexpr int kMaxPW = kMaxW + 1;    // words of P (degree 4096)

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

// A member's x-part (Section 2): w-bit words, lags r > s, shifts a..d.
struct Member {
  int w, r, s, a, b, c, d;
  int n() const { return w * r; }
};

constexpr Member kMembers[3] = {
    {32, 128, 65, 15, 14, 12, 17},  // XG_FAMILY_R128_W32 (Section 2's parameter set)
    {32, 64, 33, 19, 19, 9, 18},    // XG_FAMILY_R64_W32
    {64, 64, 33, 24, 22, 37, 45},   // XG_FAMILY_R64_W64
};

// Host stepping of a member's x-part from a fixed non-zero ring; writes bit 0
// of x_0 .. x_{nbits-1}.  Words are held in 64 bits and masked to w bits.
void xpart_bit0(const Member &m, std::vector<uint8_t> &bits) {
  const uint64_t mask = m.w == 64 ? ~0ull : (1ull << m.w) - 1;
  std::vector<uint64_t> ring((size_t)m.r);
  for (int i = 0; i < m.r; ++i) ring[(size_t)i] = (0x9E3779B97F4A7C15ull * (uint64_t)(i + 1) ^ ((uint64_t)i << 7)) & mask;
  int head = 0;  // slot of x_{k-r}
  for (size_t k = 0; k < bits.size(); ++k) {
    const uint64_t xr = ring[(size_t)head], xs = ring[(size_t)((head + m.r - m.s) % m.r)];  // x_{k-r}, x_{k-s}
    uint64_t t = xr ^ ((xr << m.a) & mask);
    t ^= t >> m.b;
    uint64_t v = xs ^ ((xs << m.c) & mask);
    v ^= v >> m.d;
    const uint64_t x = t ^ v;
    ring[(size_t)head] = x;
    head = (head + 1) % m.r;
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
  int deg = 0, w = 0, pw = 0;   // n, words of a residue, words of P
  uint64_t P[kMaxPW];
  uint64_t mu[kMaxPW];          // floor(z^(2n) / P)
  bool ok = false;
};

Modulus g_mod[3];
std::once_flag g_once[3];

void init_modulus(int f) {
  const Member &m = kMembers[f];
  Modulus &M = g_mod[f];
  const int n = m.n();
  M.deg = n;
  M.w = n / 64;
  M.pw = M.w + 1;
  std::vector<uint8_t> bits((size_t)(2 * n + 128));
  xpart_bit0(m, bits);
  std::vector<uint64_t> poly;
  if (min_poly(bits, poly) != n || poly.size() != (size_t)M.pw) return;
  std::memset(M.P, 0, sizeof(M.P));
  std::memcpy(M.P, poly.data(), sizeof(uint64_t) * (size_t)M.pw);
  // mu by long division of z^(2n) by P
  std::vector<uint64_t> rem((size_t)(2 * M.pw + 1), 0);
  rem[(size_t)(2 * n) / 64] |= 1ull << ((2 * n) % 64);
  std::memset(M.mu, 0, sizeof(M.mu));
  for (int i = 2 * n; i >= n; --i) {
    if (!((rem[(size_t)i / 64] >> (i % 64)) & 1u)) continue;
    M.mu[(i - n) / 64] |= 1ull << ((i - n) % 64);
    const int sh = i - n;
    for (int j = 0; j <= n; ++j)
      if ((M.P[j / 64] >> (j % 64)) & 1u) rem[(size_t)(j + sh) / 64] ^= 1ull << ((j + sh) % 64);
  }
  M.ok = true;
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
void mulmod(const Modulus &M, const uint64_t *a, const uint64_t *b, uint64_t *out) {
  uint64_t prod[2 * kMaxW], h[kMaxPW], t[2 * kMaxPW], q[kMaxPW], qp[2 * kMaxPW];
  pmul(a, M.w, b, M.w, prod);
  shr(prod, 2 * M.w, M.deg, h, M.pw);
  pmul(h, M.pw, M.mu, M.pw, t);
  shr(t, 2 * M.pw, M.deg, q, M.pw);
  pmul(q, M.pw, M.P, M.pw, qp);
  for (int i = 0; i < M.w; ++i) out[i] = prod[i] ^ qp[i];
}

}  // namespace

int member_degree(uint32_t family) { return family < 3 ? kMembers[family].n() : 0; }

bool jump_polynomial(uint32_t family, uint64_t J, uint64_t *g) {
  if (family >= 3) return false;
  try {
    std::call_once(g_once[family], init_modulus, (int)family);
  } catch (const std::bad_alloc &) {  // the once-flag stays unset: a later call retries
    return false;
  }
  const Modulus &M = g_mod[family];
  if (!M.ok) return false;
  uint64_t base[kMaxW] = {0}, acc[kMaxW] = {0}, tmp[kMaxW];
  base[0] = 2;  // z
  acc[0] = 1;
  const size_t bytes = sizeof(uint64_t) * (size_t)M.w;
  while (J) {
    if (J & 1u) {
      mulmod(M, acc, base, tmp);
      std::memcpy(acc, tmp, bytes);
    }
    J >>= 1;
    if (J) {
      mulmod(M, base, base, tmp);
      std::memcpy(base, tmp, bytes);
    }
  }
  std::memcpy(g, acc, bytes);
  return true;
}

bool jump_polynomial(uint64_t J, uint64_t g[64]) { return jump_polynomial(XG_FAMILY_R128_W32, J, g); }

}  // namespace xg
