// Write-only reference kernel of libxg: fills a buffer with one 32-bit value
// using 16-byte stores, so the HBM write bandwidth of the generators can be
// compared with the store path alone.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xg_internal.h"
#include "xg_launch.h"

namespace xg {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Thread i of the grid writes quad i (one 16-byte store), so block b writes
// the 4 KB piece [256 b, 256 (b + 1)); blocks are dispatched in order and the
// written region advances as one narrow front.  The words % 4 tail words are
// written by the first threads of block 0.  (Measured: 4 KB pieces and plain
// stores reach the practical ceiling; 8-16 KB pieces or non-temporal stores
// are 2-15 % slower.)
__global__ __launch_bounds__(256) void k_fill_value(uint32_t *__restrict__ out, uint64_t quads, uint32_t tail,
                                                    uint32_t value) {
  const u32x4 v = {value, value, value, value};
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i < quads) reinterpret_cast<u32x4 *>(out)[i] = v;
  if (blockIdx.x == 0 && threadIdx.x < tail) out[4 * quads + threadIdx.x] = value;
}

}  // namespace

hipError_t launch_fill_value(uint32_t *out, uint64_t words, uint32_t value, int num_cus, hipStream_t stream) {
  hipError_t e = hipSuccess;
  (void)num_cus;
  const uint64_t quads = words / 4;
  const uint64_t blocks = quads ? (quads + 255) / 256 : 1;
  if (blocks > 0xFFFFFFFFull) return hipErrorInvalidValue;
  e = launch(k_fill_value, dim3((uint32_t)blocks), dim3(256), 0, stream, out, quads, (uint32_t)(words % 4),
                     value);
  return e;
}

}  // namespace xg
