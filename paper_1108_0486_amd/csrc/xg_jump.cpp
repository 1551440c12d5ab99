// Host side of jump-ahead (libxg): the characteristic polynomial P of each
// family member's x-part step and the jump polynomials z^J mod P.
//
// The x-part of xorgens is GF(2)-linear (Section 1.5 / Section 2 of
// arXiv:1108.0486): its n-bit state S (n = r w) moves by a fixed matrix T.
// By Cayley-Hamilton T^J = g(T) with g = z^J mod P, deg g < n; the device
// evaluates g(T) on a stream's state.
//
// Everything here is linear algebra over GF(2) on n-bit vectors:
//   P      the first linear dependency among the Krylov vectors
//          S_0, T S_0, ..., T^n S_0 of a fixed non-zero start state, found by
//          Gauss-Jordan elimination (rank n means S_0 is cyclic and P is the
//          characteristic polynomial; a primitive P makes every non-zero S_0
//          cyclic).  T^k S_0 is the ring window after k host steps.
//   z^J    left-to-right binary powering in the residue ring GF(2)[z] / P, in
//          which squaring is the linear Frobenius map a -> a^2: a table of
//          z^(2i) mod P turns a square into the XOR of the entries of a's set
//          bits, and a multiplication by z is a shift with one conditional XOR
//          of P.
//   z^(kL) the server's jump table: multiplication by the fixed residue
//          h = z^L mod P is linear too; its table z^i h mod P (i < n) gives
//          each next entry as one table application.
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "xg_host.h"

namespace xg {
namespace {

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

inline bool bit_of(const uint64_t *v, int i) { return (v[i >> 6] >> (i & 63)) & 1u; }

inline void xor_into(uint64_t *dst, const uint64_t *src, int words) {
  for (int k = 0; k < words; ++k) dst[k] ^= src[k];
}

// The residue ring of one member: P, and the Frobenius table.
struct Field {
  int n = 0, words = 0;           // degree, 64-bit words of a residue
  std::vector<uint64_t> low;      // P - z^n (the bits below the leading one)
  std::vector<uint64_t> sq;       // row i: z^(2 i) mod P, i < n
  bool ok = false;

  // a <- z a mod P.
  void times_z(uint64_t *a) const {
    const bool top = bit_of(a, n - 1);
    for (int k = words - 1; k > 0; --k) a[k] = (a[k] << 1) | (a[k - 1] >> 63);
    a[0] <<= 1;
    if (top) xor_into(a, low.data(), words);
  }

  // out <- a^2 mod P (out != a).
  void square(const uint64_t *a, uint64_t *out) const {
    std::memset(out, 0, sizeof(uint64_t) * (size_t)words);
    for (int k = 0; k < words; ++k)
      for (uint64_t m = a[k]; m; m &= m - 1) {
        const int i = 64 * k + __builtin_ctzll(m);
        xor_into(out, sq.data() + (size_t)i * words, words);
      }
  }
};

Field g_field[3];
std::once_flag g_once[3];

// The member's x-part words x_{-r} .. x_{count-r-1} from a fixed non-zero
// ring, by the recurrence of Section 2 (words kept in 64 bits, masked to w).
std::vector<uint64_t> xpart_words(const Member &m, int count) {
  const uint64_t mask = m.w == 64 ? ~0ull : (1ull << m.w) - 1;
  std::vector<uint64_t> x((size_t)count);
  uint64_t z = 0x243F6A8885A308D3ull;  // any non-zero start ring will do
  for (int i = 0; i < m.r; ++i) {
    z ^= z << 13;
    z ^= z >> 7;
    z ^= z << 17;
    x[(size_t)i] = z & mask;
  }
  for (int k = m.r; k < count; ++k) {
    const uint64_t xr = x[(size_t)(k - m.r)], xs = x[(size_t)(k - m.s)];
    uint64_t t = xr ^ ((xr << m.a) & mask);
    t ^= t >> m.b;
    uint64_t v = xs ^ ((xs << m.c) & mask);
    v ^= v >> m.d;
    x[(size_t)k] = t ^ v;
  }
  return x;
}

// P from the Krylov vectors: column k (k = 0 .. n) of an n x (n + 1) bit
// matrix is S_k = (x_{k-r}, .., x_{k-1}) with bit j of word t at row t w + j.
// Gauss-Jordan on columns 0 .. n-1 leaves, at full rank, column n equal to
// the coefficients c with S_n = sum_k c_k S_k, so P = z^n + sum_k c_k z^k.
bool derive_p(const Member &m, Field &F) {
  const int n = m.n(), cols = n + 1, rw = (cols + 63) / 64;
  const std::vector<uint64_t> x = xpart_words(m, n + m.r);  // x[i] = x_{i-r}
  std::vector<uint64_t> rows((size_t)n * rw, 0);
  for (int b = 0; b < n; ++b) {
    const int t = b / m.w, j = b % m.w;
    uint64_t *row = rows.data() + (size_t)b * rw;
    for (int k = 0; k < cols; ++k)
      if ((x[(size_t)(k + t)] >> j) & 1u) row[k >> 6] |= 1ull << (k & 63);
  }
  for (int col = 0; col < n; ++col) {
    int piv = -1;
    for (int i = col; i < n; ++i)
      if (bit_of(rows.data() + (size_t)i * rw, col)) {
        piv = i;
        break;
      }
    if (piv < 0) return false;  // rank below n: not the characteristic polynomial
    uint64_t *pr = rows.data() + (size_t)piv * rw;
    if (piv != col) {
      uint64_t *cr = rows.data() + (size_t)col * rw;
      for (int k = 0; k < rw; ++k) std::swap(pr[k], cr[k]);
      pr = cr;
    }
    const int from = col >> 6;  // the pivot row is zero left of col
    for (int i = 0; i < n; ++i) {
      if (i == col) continue;
      uint64_t *ri = rows.data() + (size_t)i * rw;
      if (bit_of(ri, col)) xor_into(ri + from, pr + from, rw - from);
    }
  }
  F.n = n;
  F.words = n / 64;
  F.low.assign((size_t)F.words, 0);
  for (int k = 0; k < n; ++k)
    if (bit_of(rows.data() + (size_t)k * rw, n)) F.low[(size_t)k >> 6] |= 1ull << (k & 63);
  return true;
}

void build_field(int f) {
  Field &F = g_field[f];
  if (!derive_p(kMembers[f], F)) return;
  const int n = F.n, W = F.words;
  F.sq.assign((size_t)n * W, 0);
  std::vector<uint64_t> cur((size_t)W, 0);
  cur[0] = 1;
  for (int i = 0; i < n; ++i) {  // row i = z^(2 i) mod P
    std::memcpy(F.sq.data() + (size_t)i * W, cur.data(), sizeof(uint64_t) * (size_t)W);
    F.times_z(cur.data());
    F.times_z(cur.data());
  }
  F.ok = true;
}

const Field *field(uint32_t family) {
  if (family >= 3) return nullptr;
  try {
    std::call_once(g_once[family], build_field, (int)family);
  } catch (const std::bad_alloc &) {  // the once-flag stays unset: a later call retries
    return nullptr;
  }
  return g_field[family].ok ? &g_field[family] : nullptr;
}

// g <- z^J mod P: for the bits of J from the top, g <- g^2, then g <- z g
// where the bit is set.
void z_pow(const Field &F, uint64_t J, uint64_t *g) {
  std::memset(g, 0, sizeof(uint64_t) * (size_t)F.words);
  g[0] = 1;
  if (J == 0) return;
  std::vector<uint64_t> tmp((size_t)F.words);
  for (int b = 63 - __builtin_clzll(J); b >= 0; --b) {
    F.square(g, tmp.data());
    std::memcpy(g, tmp.data(), sizeof(uint64_t) * (size_t)F.words);
    if ((J >> b) & 1u) F.times_z(g);
  }
}

// The most recently used jump polynomials, least recently used replaced.
struct CachedJump {
  uint32_t family = 0;
  uint64_t J = 0;
  uint64_t used = 0;  // 0: empty
  std::vector<uint64_t> g;
};
constexpr size_t kCachedJumps = 16;
std::mutex g_cache_mu;
CachedJump g_cache[kCachedJumps];
uint64_t g_cache_clock = 0;

}  // namespace

int member_degree(uint32_t family) { return family < 3 ? kMembers[family].n() : 0; }

bool jump_polynomial_uncached(uint32_t family, uint64_t J, uint64_t *g) {
  const Field *F = field(family);
  if (!F) return false;
  try {
    z_pow(*F, J, g);
  } catch (const std::bad_alloc &) {
    return false;
  }
  return true;
}

bool jump_polynomial(uint32_t family, uint64_t J, uint64_t *g) {
  const Field *F = field(family);
  if (!F) return false;
  const size_t words = (size_t)F->words;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (CachedJump &e : g_cache)
      if (e.used && e.family == family && e.J == J) {
        std::memcpy(g, e.g.data(), sizeof(uint64_t) * words);
        e.used = ++g_cache_clock;
        return true;
      }
  }
  if (!jump_polynomial_uncached(family, J, g)) return false;
  try {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    CachedJump *slot = &g_cache[0];
    for (CachedJump &e : g_cache)
      if (e.used < slot->used) slot = &e;  // an empty entry (0) first, else the oldest
    slot->g.assign(g, g + words);
    slot->family = family;
    slot->J = J;
    slot->used = ++g_cache_clock;
  } catch (const std::bad_alloc &) {  // the result stands; it is only not kept
  }
  return true;
}

bool jump_polynomial(uint64_t J, uint64_t g[64]) { return jump_polynomial(XG_FAMILY_R128_W32, J, g); }

bool jump_table(uint32_t family, uint64_t L, uint32_t count, uint64_t *table) {
  const Field *F = field(family);
  if (!F) return false;
  const int n = F->n, W = F->words;
  try {
    // mul row i = z^i h mod P, h = z^L mod P: multiplication by h as a table.
    std::vector<uint64_t> mul((size_t)n * W), cur((size_t)W);
    z_pow(*F, L, cur.data());
    for (int i = 0; i < n; ++i) {
      std::memcpy(mul.data() + (size_t)i * W, cur.data(), sizeof(uint64_t) * (size_t)W);
      F->times_z(cur.data());
    }
    std::vector<uint64_t> prev((size_t)W, 0);
    prev[0] = 1;  // z^0
    for (uint32_t k = 0; k < count; ++k) {
      uint64_t *out = table + (size_t)k * W;
      std::memset(out, 0, sizeof(uint64_t) * (size_t)W);
      for (int q = 0; q < W; ++q)
        for (uint64_t m = prev[(size_t)q]; m; m &= m - 1)
          xor_into(out, mul.data() + (size_t)(64 * q + __builtin_ctzll(m)) * W, W);
      std::memcpy(prev.data(), out, sizeof(uint64_t) * (size_t)W);
    }
  } catch (const std::bad_alloc &) {
    return false;
  }
  return true;
}

}  // namespace xg
