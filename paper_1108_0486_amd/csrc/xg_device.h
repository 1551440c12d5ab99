// Device helpers shared by libxg's HIP kernels (gfx950): lane rotation by
// DPP, three-input bit operations, the block numbering by XCD, and
// SplitMix64 (the seeding generator).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xg {
namespace dev {

// Lane l receives lane l-1's value, lane 0 receives lane 63's (DPP
// wave_ror:1; every lane has a valid source, so bound_ctrl never applies).
__device__ __forceinline__ uint32_t lanes_rotate_up(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x13C, 0xF, 0xF, true);
}

// A truth table of v_bitop3_b32 is the function's value on the operand
// patterns a = 0xF0, b = 0xCC, c = 0xAA.
// a xor b xor c: 0x96.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// a xor (b and m): 0xF0 ^ (0xCC & 0xAA) = 0x78.
__device__ __forceinline__ uint32_t xor_and(uint32_t a, uint32_t b, uint32_t m) {
  return __builtin_amdgcn_bitop3_b32(a, b, m, 0x78);
}

// Bits of a where m is set, of b elsewhere: (a & m) | (b & ~m), 0xE4.
__device__ __forceinline__ uint32_t select_bits(uint32_t a, uint32_t b, uint32_t m) {
  return __builtin_amdgcn_bitop3_b32(a, b, m, 0xE4);
}

// Workgroups are dispatched to MI355X's 8 XCDs in turn (block b to XCD
// b mod 8) and each XCD has its own L2.  Renumbering the first 8 floor(nb / 8)
// blocks so that XCD x gets the consecutive numbers [x nb8, (x + 1) nb8),
// nb8 = floor(nb / 8), gives each XCD a contiguous range of streams.  The map
// is a bijection; the remaining blocks keep their number.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block() {
  const uint32_t b = blockIdx.x, full = gridDim.x & ~(kXcds - 1);
  return b < full ? (b % kXcds) * (full / kXcds) + b / kXcds : b;
}

// Orders a wavefront's LDS accesses before it against those after it.  Lanes
// read words other lanes wrote; without a fence the compiler may move (or
// drop) such accesses as if each lane only ever read its own writes.  The
// fences cover LDS only, so outstanding global stores are not waited for.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// k-th output (k >= 1) of SplitMix64 (Steele, Lea & Flood 2014) started at
// s: after k increments the state is s + k * gamma, gamma the golden-ratio
// constant, then the finaliser.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t s, uint64_t k) {
  uint64_t z = s + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace dev
}  // namespace xg
