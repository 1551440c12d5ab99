// Kernel launches that report their own status.
#pragma once

#include <hip/hip_runtime.h>

#include <tuple>
#include <type_traits>
#include <utility>

namespace xg {

// Enqueues kernel<<<grid, block, lds, stream>>>(args...) through
// hipLaunchKernel and returns the status of this launch alone.  (Reading
// hipGetLastError after a launch would also return an error that an unrelated
// earlier HIP call left behind on the same host thread.)  The arguments are
// converted to the kernel's parameter types before their addresses are taken.
template <typename... P, typename... A>
inline hipError_t launch(void (*kernel)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t stream,
                         A &&...args) {
  static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
  std::tuple<std::decay_t<P>...> held(std::forward<A>(args)...);
  return std::apply(
      [&](auto &...v) {
        void *argv[] = {static_cast<void *>(&v)...};
        return hipLaunchKernel(reinterpret_cast<const void *>(kernel), grid, block, argv, lds, stream);
      },
      held);
}

// A persistent kernel's launch: at most as many blocks as num_cus compute
// units hold at once (by the runtime's occupancy for this kernel, block size
// and LDS).  Blocks beyond that would start only as resident ones exit, after
// the work is gone, and the batch kernels give each wavefront's first item by
// its index in the grid, so every wavefront must be running from the start.
template <typename... P, typename... A>
inline hipError_t launch_persistent(void (*kernel)(P...), uint64_t blocks, dim3 block, size_t lds, int num_cus,
                                    hipStream_t stream, A &&...args) {
  int per_cu = 0;
  const int threads = (int)(block.x * block.y * block.z);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kernel), threads, lds) ==
          hipSuccess &&
      per_cu > 0) {
    const uint64_t cap = (uint64_t)per_cu * (uint64_t)(num_cus > 0 ? num_cus : 1);
    if (blocks > cap) blocks = cap;
  }
  return launch(kernel, dim3((uint32_t)(blocks ? blocks : 1)), block, lds, stream, std::forward<A>(args)...);
}

}  // namespace xg
